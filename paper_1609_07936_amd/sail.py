"""Python binding of libsail (the gfx950 SAIL annealing library).

Argument marshalling only: every step of the anneal runs in the HIP
kernels behind the C ABI declared in include/sail.h.  PyTorch supplies the
HIP stream (and device buffers for the optional trace).  Importing this
module fails loudly when the built library is missing; there is no CPU
fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsail.so")

SAIL_K_POINT, SAIL_K_BIN_EXACT = 0, 1
SAIL_JOB_QUEUED, SAIL_JOB_RUNNING, SAIL_JOB_DONE = 0, 1, 2
SAIL_FP64, SAIL_FP32 = 0, 1


class SailError(RuntimeError):
    def __init__(self, status: int, what: str, message: str):
        super().__init__(f"{what}: {message} (status {status})")
        self.status = status


class ScheduleC(ctypes.Structure):
    _fields_ = [
        ("T", ctypes.c_void_p), ("n_T", ctypes.c_int),
        ("branch_every", ctypes.c_int), ("resync_every", ctypes.c_int),
        ("branch_fraction", ctypes.c_double), ("imprint_t", ctypes.c_double),
        ("eps0", ctypes.c_double), ("amp_p", ctypes.c_double), ("amp_m", ctypes.c_int),
        ("amp_avg", ctypes.c_double), ("walk_len", ctypes.c_int), ("t_units", ctypes.c_int),
        ("smooth", ctypes.c_double), ("adaptive", ctypes.c_int),
        ("self_cool", ctypes.c_int), ("boil_blocks", ctypes.c_int), ("cool_blocks", ctypes.c_int),
    ]


class JobC(ctypes.Structure):
    _fields_ = [
        ("omega", ctypes.c_void_p), ("n_omega", ctypes.c_int),
        ("tau", ctypes.c_void_p), ("n_tau", ctypes.c_int),
        ("F", ctypes.c_void_p), ("sigma", ctypes.c_void_p),
        ("m0", ctypes.c_double), ("m1", ctypes.c_double),
        ("kernel_mode", ctypes.c_int),
        ("n_walkers", ctypes.c_int), ("seed", ctypes.c_uint64), ("precision", ctypes.c_int),
        ("tau_per_lane", ctypes.c_int),
        ("sched", ScheduleC),
    ]


class ServerConfigC(ctypes.Structure):
    _fields_ = [("device", ctypes.c_int), ("hbm_bytes", ctypes.c_size_t), ("max_jobs", ctypes.c_int)]


class JobResultC(ctypes.Structure):
    _fields_ = [
        ("status", ctypes.c_int),
        ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double), ("t_done", ctypes.c_double),
        ("chi2_unit", ctypes.c_double), ("chi2_min", ctypes.c_double), ("chi2_median", ctypes.c_double),
        ("n_omega", ctypes.c_int), ("n_walkers", ctypes.c_int),
    ]


class BlockRecordC(ctypes.Structure):
    _fields_ = [("sweep", ctypes.c_int32), ("event", ctypes.c_int32), ("T", ctypes.c_double),
                ("chi2_min", ctypes.c_double), ("chi2_mean", ctypes.c_double), ("chi2_median", ctypes.c_double),
                ("chi2_max", ctypes.c_double),
                ("rate_mean", ctypes.c_double), ("drift_max", ctypes.c_double)]


class ServerStatsC(ctypes.Structure):
    _fields_ = [
        ("submitted", ctypes.c_int64), ("admitted", ctypes.c_int64), ("completed", ctypes.c_int64),
        ("failed", ctypes.c_int64), ("queued", ctypes.c_int), ("in_flight", ctypes.c_int),
        ("arena_bytes", ctypes.c_size_t), ("arena_used", ctypes.c_size_t), ("arena_peak", ctypes.c_size_t),
        ("rounds", ctypes.c_int64), ("sweep_ms", ctypes.c_double), ("sweep_launches", ctypes.c_int64),
        ("cancelled", ctypes.c_int64),
    ]


_lib = None

_ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p)
_FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p)
# Every pair of callbacks ever installed stays referenced: blocks go back to
# the allocator that made them, also after the hook has changed.
_installed_hooks: list = []


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libsail.so is not built ({LIB_PATH}); run __graft_entry__.build() first")
    L = ctypes.CDLL(LIB_PATH)
    P, I, D = ctypes.c_void_p, ctypes.c_int, ctypes.c_double
    st = ctypes.c_int
    L.sail_schedule_defaults.argtypes = [ctypes.POINTER(ScheduleC)]
    L.sail_schedule_defaults.restype = None
    L.sail_problem_create.argtypes = [P, I, P, I, P, P, D, D, I, I, ctypes.POINTER(P)]
    L.sail_problem_create.restype = st
    L.sail_problem_destroy.argtypes = [P]
    L.sail_problem_destroy.restype = None
    L.sail_walkers_init.argtypes = [P, I, ctypes.c_uint64, I, P]
    L.sail_walkers_init.restype = st
    L.sail_run_schedule.argtypes = [P, ctypes.POINTER(ScheduleC), I, I, P]
    L.sail_run_schedule.restype = st
    L.sail_chi2_unit.argtypes = [P]
    L.sail_chi2_unit.restype = D
    L.sail_read_spectrum.argtypes = [P, P, P]
    L.sail_read_spectrum.restype = st
    L.sail_read_chi2.argtypes = [P, P, P]
    L.sail_read_chi2.restype = st
    L.sail_read_chi2_hist.argtypes = [P, I, D, D, P, P]
    L.sail_read_chi2_hist.restype = st
    L.sail_read_chi2_hist_noalloc.argtypes = [P, I, D, D, P, P]
    L.sail_read_chi2_hist_noalloc.restype = st
    L.sail_read_state.argtypes = [P, P, P, P, P]
    L.sail_read_state.restype = st
    L.sail_read_events.argtypes = [P, I, P, P, P, P, P]
    L.sail_read_events.restype = st
    L.sail_set_watchdog.argtypes = [P, D]
    L.sail_set_watchdog.restype = st
    L.sail_watchdog_report.argtypes = [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.sail_watchdog_report.restype = st
    L.sail_set_block_log.argtypes = [P, I]
    L.sail_set_block_log.restype = st
    L.sail_read_block_log.argtypes = [P, ctypes.POINTER(BlockRecordC), I, ctypes.POINTER(ctypes.c_int),
                                      ctypes.POINTER(ctypes.c_int64), P]
    L.sail_read_block_log.restype = st
    L.sail_read_event_margins.argtypes = [P, I, P, P]
    L.sail_read_event_margins.restype = st
    L.sail_set_event_log.argtypes = [P, I]
    L.sail_set_event_log.restype = st
    L.sail_set_trace.argtypes = [P, I, I, P, P]
    L.sail_set_trace.restype = st
    L.sail_set_timing.argtypes = [P, I]
    L.sail_set_timing.restype = st
    L.sail_sweep_timing.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), I]
    L.sail_sweep_timing.restype = st
    L.sail_footprint_bytes.argtypes = [I, I, I, I]
    L.sail_footprint_bytes.restype = ctypes.c_size_t
    L.sail_layout.argtypes = [P, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]
    L.sail_layout.restype = st
    L.sail_state_export.argtypes = [P, P, ctypes.POINTER(ctypes.c_size_t), P]
    L.sail_state_export.restype = st
    L.sail_state_import.argtypes = [P, P, ctypes.c_size_t, P]
    L.sail_state_import.restype = st
    L.sail_set_tau_per_lane.argtypes = [P, I]
    L.sail_set_tau_per_lane.restype = st
    L.sail_autotune_layout.argtypes = [P, I, I, ctypes.POINTER(ctypes.c_int), P]
    L.sail_autotune_layout.restype = st
    L.sail_autotune_layout_alone.argtypes = [P, I, I, ctypes.POINTER(ctypes.c_int), P]
    L.sail_autotune_layout_alone.restype = st
    L.sail_batch_create.argtypes = [ctypes.POINTER(P), I, ctypes.POINTER(P)]
    L.sail_batch_create.restype = st
    L.sail_batch_destroy.argtypes = [P]
    L.sail_batch_destroy.restype = None
    L.sail_batch_run.argtypes = [P, ctypes.POINTER(ctypes.POINTER(ScheduleC)), P, P, P]
    L.sail_batch_run.restype = st
    L.sail_batch_set_timing.argtypes = [P, I]
    L.sail_batch_set_timing.restype = st
    L.sail_batch_sweep_timing.argtypes = [P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int64), I]
    L.sail_batch_sweep_timing.restype = st
    L.sail_server_create.argtypes = [ctypes.POINTER(ServerConfigC), ctypes.POINTER(P)]
    L.sail_server_create.restype = st
    L.sail_server_submit.argtypes = [P, ctypes.POINTER(JobC), ctypes.POINTER(ctypes.c_int64)]
    L.sail_server_submit.restype = st
    L.sail_server_wait.argtypes = [P, ctypes.c_int64, D, ctypes.POINTER(JobResultC), P]
    L.sail_server_wait.restype = st
    L.sail_server_poll.argtypes = [P, ctypes.c_int64, ctypes.POINTER(ctypes.c_int)]
    L.sail_server_poll.restype = st
    L.sail_server_cancel.argtypes = [P, ctypes.c_int64]
    L.sail_server_cancel.restype = st
    L.sail_server_get_stats.argtypes = [P, ctypes.POINTER(ServerStatsC)]
    L.sail_server_get_stats.restype = st
    L.sail_server_clock.argtypes = [P]
    L.sail_server_clock.restype = D
    L.sail_job_footprint_bytes.argtypes = [ctypes.POINTER(JobC)]
    L.sail_job_footprint_bytes.restype = ctypes.c_size_t
    L.sail_server_destroy.argtypes = [P]
    L.sail_server_destroy.restype = None
    L.sail_set_allocator.argtypes = [_ALLOC_FN, _FREE_FN, P]
    L.sail_set_allocator.restype = st
    L.sail_status_string.argtypes = [I]
    L.sail_status_string.restype = ctypes.c_char_p
    L.sail_last_error.argtypes = []
    L.sail_last_error.restype = ctypes.c_char_p
    _lib = L
    return L


def _check(status: int, what: str) -> None:
    if status != 0:
        msg = lib().sail_last_error().decode(errors="replace")
        raise SailError(status, what, msg or lib().sail_status_string(status).decode())


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


def _stream_handle(stream) -> int | None:
    """A HIP stream handle: an int, a torch.cuda.Stream, or None for torch's
    current stream (the null stream without torch)."""
    if stream is None:
        try:
            import torch
            if torch.cuda.is_available():
                return int(torch.cuda.current_stream().cuda_stream) or None
        except Exception:
            return None
        return None
    if isinstance(stream, int):
        return stream or None
    return int(stream.cuda_stream) or None


def set_allocator(alloc=None, release=None) -> None:
    """Routes the library's device allocations through alloc(bytes, device)
    -> int address (0 or None when out of memory) and release(address, bytes,
    device); both None restores hipMalloc/hipFree.  Process-wide."""
    if (alloc is None) != (release is None):
        raise ValueError("give both functions or neither")
    if alloc is None:
        _check(lib().sail_set_allocator(_ALLOC_FN(), _FREE_FN(), None), "sail_set_allocator")
        return

    def _a(nbytes, device, _user):
        try:
            return int(alloc(int(nbytes), int(device)) or 0) or None
        except Exception:
            return None

    def _r(ptr, nbytes, device, _user):
        try:
            release(int(ptr), int(nbytes), int(device))
        except Exception:  # e.g. at interpreter exit, with the allocator already torn down
            pass

    pair = (_ALLOC_FN(_a), _FREE_FN(_r))
    _installed_hooks.append(pair)
    # the library may call these for blocks it still holds while the
    # interpreter shuts down, after this module's globals are gone: keep the
    # two thunks alive for the life of the process
    for cb in pair:
        ctypes.pythonapi.Py_IncRef(ctypes.py_object(cb))
    _check(lib().sail_set_allocator(pair[0], pair[1], None), "sail_set_allocator")


def use_torch_allocator(enable: bool = True) -> None:
    """Takes the library's device buffers from PyTorch's caching allocator
    (enable=False goes back to hipMalloc).  Blocks are allocated on torch's
    current stream of the device; the library synchronises the device before
    it hands one back."""
    if not enable:
        set_allocator(None, None)
        return
    import torch

    def alloc(nbytes, device):
        return torch.cuda.caching_allocator_alloc(nbytes, device=device)

    def release(ptr, _nbytes, _device):
        torch.cuda.caching_allocator_delete(ptr)

    set_allocator(alloc, release)


def footprint_bytes(n_omega: int, n_tau: int, n_walkers: int, precision: int = SAIL_FP64) -> int:
    return int(lib().sail_footprint_bytes(n_omega, n_tau, n_walkers, precision))


class Schedule:
    """Annealing schedule; defaults are those of Sec. 3 of the paper plus the
    running-average weight of the acceptance rate."""

    def __init__(self, T, branch_every=100, resync_every=100, branch_fraction=0.25, imprint_t=0.1, eps0=0.1,
                 amp_p=1.0, amp_m=2, amp_avg=0.1, walk_len=0, t_units=0, smooth=0.0,
                 adaptive=0, self_cool=0, boil_blocks=0, cool_blocks=1):
        self.T = _f64(T)
        self.c = ScheduleC()
        lib().sail_schedule_defaults(ctypes.byref(self.c))
        c = self.c
        c.T, c.n_T = _p(self.T), self.T.size
        c.branch_every, c.resync_every = int(branch_every), int(resync_every)
        c.branch_fraction, c.imprint_t, c.eps0 = float(branch_fraction), float(imprint_t), float(eps0)
        c.amp_p, c.amp_m, c.amp_avg = float(amp_p), int(amp_m), float(amp_avg)
        c.walk_len, c.t_units = int(walk_len), int(t_units)
        c.smooth = float(smooth)
        c.adaptive = int(adaptive)
        c.self_cool, c.boil_blocks, c.cool_blocks = int(self_cool), int(boil_blocks), int(cool_blocks)

    @property
    def n_sweeps(self) -> int:
        return int(self.T.size)


class Problem:
    """One inversion on one GPU (see sail_problem_create)."""

    def __init__(self, omega, tau, F, sigma, m0: float, m1: float, mode: int = SAIL_K_POINT, device: int = 0):
        self.omega, self.tau, self.F = _f64(omega), _f64(tau), _f64(F)
        self.sigma = None if sigma is None else _f64(sigma)
        self.n_omega, self.n_tau = self.omega.size, self.tau.size
        self.n_walkers = 0
        h = ctypes.c_void_p()
        _check(lib().sail_problem_create(_p(self.omega), self.n_omega, _p(self.tau), self.n_tau, _p(self.F),
                                         _p(self.sigma), float(m0), float(m1), int(mode), int(device),
                                         ctypes.byref(h)), "sail_problem_create")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().sail_problem_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_walkers(self, n_walkers: int, seed: int, precision: int = SAIL_FP64, stream=None) -> float:
        _check(lib().sail_walkers_init(self._h, int(n_walkers), int(seed), int(precision), _stream_handle(stream)),
               "sail_walkers_init")
        self.n_walkers = int(n_walkers)
        return self.chi2_unit

    @property
    def chi2_unit(self) -> float:
        return float(lib().sail_chi2_unit(self._h))

    def run(self, sched: Schedule, first_sweep: int, n_sweeps: int, stream=None) -> None:
        _check(lib().sail_run_schedule(self._h, ctypes.byref(sched.c), int(first_sweep), int(n_sweeps),
                                       _stream_handle(stream)), "sail_run_schedule")

    def read_spectrum(self, stream=None) -> np.ndarray:
        out = np.zeros(self.n_omega)
        _check(lib().sail_read_spectrum(self._h, _p(out), _stream_handle(stream)), "sail_read_spectrum")
        return out

    def read_chi2(self, stream=None) -> np.ndarray:
        out = np.zeros(self.n_walkers)
        _check(lib().sail_read_chi2(self._h, _p(out), _stream_handle(stream)), "sail_read_chi2")
        return out

    def read_chi2_hist(self, n_bins: int = 64, lo: float = float("nan"), hi: float = float("nan"),
                       stream=None) -> np.ndarray:
        out = np.zeros(n_bins, dtype=np.uint64)
        _check(lib().sail_read_chi2_hist(self._h, int(n_bins), float(lo), float(hi), _p(out),
                                         _stream_handle(stream)), "sail_read_chi2_hist")
        return out

    def read_chi2_hist_noalloc(self, n_bins: int = 64, lo: float = float("nan"), hi: float = float("nan"),
                               out_ptr: int | None = None, stream=None) -> np.ndarray | None:
        """The histogram through the entry point that allocates no device
        memory.  With out_ptr (an address of n_bins uint64, host or device)
        the counts go there and None is returned."""
        out = None if out_ptr is not None else np.zeros(n_bins, dtype=np.uint64)
        dst = ctypes.c_void_p(out_ptr) if out_ptr is not None else _p(out)
        _check(lib().sail_read_chi2_hist_noalloc(self._h, int(n_bins), float(lo), float(hi), dst,
                                                 _stream_handle(stream)), "sail_read_chi2_hist_noalloc")
        return out

    def read_state(self, stream=None) -> dict:
        a = np.zeros((self.n_walkers, self.n_omega))
        F = np.zeros((self.n_walkers, self.n_tau))
        rate = np.zeros(self.n_walkers)
        _check(lib().sail_read_state(self._h, _p(a), _p(F), _p(rate), _stream_handle(stream)), "sail_read_state")
        return {"a": a, "F": F, "rate": rate}

    def set_watchdog(self, drift_bound: float) -> None:
        _check(lib().sail_set_watchdog(self._h, float(drift_bound)), "sail_set_watchdog")

    def watchdog_report(self) -> tuple[int, int]:
        """(sweep after which the last call's check tripped, sweep restored to); -1, -1 if none."""
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(lib().sail_watchdog_report(self._h, ctypes.byref(a), ctypes.byref(b)), "sail_watchdog_report")
        return a.value, b.value

    def set_block_log(self, capacity: int) -> None:
        _check(lib().sail_set_block_log(self._h, int(capacity)), "sail_set_block_log")

    def read_block_log(self, max_records: int = 1 << 20, stream=None) -> dict:
        """The newest records of the per-block log, oldest first, as arrays
        keyed by field, plus 'total' (records appended since the log was
        switched on)."""
        n = ctypes.c_int()
        total = ctypes.c_int64()
        probe = (BlockRecordC * 1)()
        _check(lib().sail_read_block_log(self._h, probe, 0, ctypes.byref(n), ctypes.byref(total),
                                         _stream_handle(stream)), "sail_read_block_log")
        m = int(min(max_records, total.value))
        buf = (BlockRecordC * max(m, 1))()
        _check(lib().sail_read_block_log(self._h, buf, m, ctypes.byref(n), ctypes.byref(total),
                                         _stream_handle(stream)), "sail_read_block_log")
        recs = buf[:n.value]
        out = {f: np.array([getattr(r, f) for r in recs]) for f, _ in BlockRecordC._fields_}
        out["total"] = total.value
        return out

    def set_event_log(self, keep_multipliers: bool) -> None:
        _check(lib().sail_set_event_log(self._h, int(bool(keep_multipliers))), "sail_set_event_log")

    def read_events(self, n_events: int, multipliers: bool = False) -> dict:
        d = np.zeros(n_events)
        pr = np.zeros(n_events)
        z = np.zeros(n_events, dtype=np.int32)
        stt = np.zeros(n_events, dtype=np.int32)
        m = np.zeros((n_events, self.n_walkers), dtype=np.int32) if multipliers else None
        _check(lib().sail_read_events(self._h, int(n_events), _p(d), _p(pr), _p(z), _p(stt), _p(m)),
               "sail_read_events")
        out = {"delta": d, "pr": pr, "z": z, "status": stt}
        if multipliers:
            out["m"] = m
        gap, bracket = np.zeros(n_events), np.zeros(n_events)
        _check(lib().sail_read_event_margins(self._h, int(n_events), _p(gap), _p(bracket)), "sail_read_event_margins")
        out["gap"], out["bracket"] = gap, bracket
        return out

    def set_trace(self, k0: int, k1: int, dchi2_ptr: int = 0, flags_ptr: int = 0) -> None:
        """Device buffers [n_walkers][k1 - k0][n_omega] (float64 and uint8)."""
        _check(lib().sail_set_trace(self._h, int(k0), int(k1), ctypes.c_void_p(dchi2_ptr or None),
                                    ctypes.c_void_p(flags_ptr or None)), "sail_set_trace")

    def set_timing(self, enable: bool) -> None:
        _check(lib().sail_set_timing(self._h, int(bool(enable))), "sail_set_timing")

    def sweep_timing(self, reset: bool = False) -> tuple[float, int]:
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().sail_sweep_timing(self._h, ctypes.byref(ms), ctypes.byref(n), int(bool(reset))),
               "sail_sweep_timing")
        return ms.value, n.value

    def state_export(self, stream=None) -> bytes:
        n = ctypes.c_size_t(0)
        _check(lib().sail_state_export(self._h, None, ctypes.byref(n), _stream_handle(stream)), "sail_state_export")
        buf = ctypes.create_string_buffer(n.value)
        _check(lib().sail_state_export(self._h, buf, ctypes.byref(n), _stream_handle(stream)), "sail_state_export")
        return buf.raw[:n.value]

    def state_import(self, blob: bytes, stream=None) -> None:
        buf = ctypes.create_string_buffer(blob, len(blob))
        _check(lib().sail_state_import(self._h, buf, len(blob), _stream_handle(stream)), "sail_state_import")

    def set_tau_per_lane(self, tpl: int) -> None:
        _check(lib().sail_set_tau_per_lane(self._h, int(tpl)), "sail_set_tau_per_lane")

    def autotune_layout(self, n_walkers: int, precision: int = SAIL_FP64, stream=None, alone: bool = False) -> int:
        """Times the candidate lane layouts and requests the fastest for the
        next init_walkers (this leaves the problem without walkers); alone:
        the problem has the device to itself, so the smallest tile is a
        candidate too."""
        v = ctypes.c_int()
        fn, name = ((lib().sail_autotune_layout_alone, "sail_autotune_layout_alone") if alone
                    else (lib().sail_autotune_layout, "sail_autotune_layout"))
        _check(fn(self._h, int(n_walkers), int(precision), ctypes.byref(v), _stream_handle(stream)), name)
        self.n_walkers = 0
        return v.value

    def layout(self) -> tuple[int, int]:
        a, b = ctypes.c_int(), ctypes.c_int()
        _check(lib().sail_layout(self._h, ctypes.byref(a), ctypes.byref(b)), "sail_layout")
        return a.value, b.value


class Batch:
    """Many problems annealed together (see sail_batch_create); the batch
    refers to the problems, which must stay alive while it is used."""

    def __init__(self, problems):
        self.problems = list(problems)
        arr = (ctypes.c_void_p * len(self.problems))(*[pr._h for pr in self.problems])
        h = ctypes.c_void_p()
        _check(lib().sail_batch_create(arr, len(self.problems), ctypes.byref(h)), "sail_batch_create")
        self._h = h

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().sail_batch_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def run(self, scheds, first_sweeps, n_sweeps, stream=None) -> None:
        """scheds: one Schedule per problem (or one for all); first_sweeps and
        n_sweeps: ints or one per problem."""
        n = len(self.problems)
        if isinstance(scheds, Schedule):
            scheds = [scheds] * n
        f = np.ascontiguousarray(np.broadcast_to(np.asarray(first_sweeps, dtype=np.int32), (n,)))
        k = np.ascontiguousarray(np.broadcast_to(np.asarray(n_sweeps, dtype=np.int32), (n,)))
        if len(scheds) != n:
            raise ValueError("one schedule per problem")
        ptrs = (ctypes.POINTER(ScheduleC) * n)(*[ctypes.pointer(sc.c) for sc in scheds])
        _check(lib().sail_batch_run(self._h, ptrs, _p(f), _p(k), _stream_handle(stream)), "sail_batch_run")

    def set_timing(self, enable: bool) -> None:
        _check(lib().sail_batch_set_timing(self._h, int(bool(enable))), "sail_batch_set_timing")

    def sweep_timing(self, reset: bool = False) -> tuple[float, int]:
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        _check(lib().sail_batch_sweep_timing(self._h, ctypes.byref(ms), ctypes.byref(n), int(bool(reset))),
               "sail_batch_sweep_timing")
        return ms.value, n.value


SAIL_ESTATE, SAIL_ETIMEOUT, SAIL_ECANCELLED = 6, 7, 8
AUTOTUNE = -1


class Server:
    """A served-anneal server on one device (see sail_server_create): jobs
    are submitted from any thread and waited for by id."""

    def __init__(self, hbm_bytes: int, max_jobs: int, device: int = 0):
        cfg = ServerConfigC(int(device), int(hbm_bytes), int(max_jobs))
        h = ctypes.c_void_p()
        _check(lib().sail_server_create(ctypes.byref(cfg), ctypes.byref(h)), "sail_server_create")
        self._h = h
        self._n_omega = {}

    def close(self) -> None:
        if getattr(self, "_h", None):
            lib().sail_server_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    @staticmethod
    def _job(omega, tau, F, sigma, m0, m1, n_walkers, seed, sched, precision, tau_per_lane, mode):
        om, ta, f = _f64(omega), _f64(tau), _f64(F)
        sg = None if sigma is None else _f64(sigma)
        job = JobC(_p(om), om.size, _p(ta), ta.size, _p(f), _p(sg), float(m0), float(m1), int(mode),
                   int(n_walkers), int(seed), int(precision), int(tau_per_lane), sched.c)
        return job, (om, ta, f, sg)

    @staticmethod
    def job_footprint(omega, tau, n_walkers, sched: Schedule, precision=SAIL_FP64) -> int:
        om, ta = _f64(omega), _f64(tau)
        job = JobC(_p(om), om.size, _p(ta), ta.size, _p(ta), None, 1.0, 0.0, 0, int(n_walkers), 0, int(precision),
                   0, sched.c)
        return int(lib().sail_job_footprint_bytes(ctypes.byref(job)))

    def submit(self, omega, tau, F, sigma, m0, m1, n_walkers, seed, sched: Schedule, precision=SAIL_FP64,
               tau_per_lane=AUTOTUNE, mode=SAIL_K_POINT) -> int:
        job, keep = self._job(omega, tau, F, sigma, m0, m1, n_walkers, seed, sched, precision, tau_per_lane, mode)
        om = keep[0]
        jid = ctypes.c_int64()
        _check(lib().sail_server_submit(self._h, ctypes.byref(job), ctypes.byref(jid)), "sail_server_submit")
        self._n_omega[jid.value] = om.size
        return jid.value

    def wait(self, job_id: int, timeout: float = -1.0) -> dict:
        mean = np.zeros(max(1, self._n_omega.get(job_id, 0)))
        r = JobResultC()
        _check(lib().sail_server_wait(self._h, int(job_id), float(timeout), ctypes.byref(r), _p(mean)),
               "sail_server_wait")
        self._n_omega.pop(job_id, None)
        out = {k: getattr(r, k) for k, _ in JobResultC._fields_}
        out["mean_spectrum"] = mean if r.status == 0 else None
        return out

    def poll(self, job_id: int) -> int:
        """SAIL_JOB_QUEUED, SAIL_JOB_RUNNING or SAIL_JOB_DONE, without waiting."""
        state = ctypes.c_int()
        _check(lib().sail_server_poll(self._h, int(job_id), ctypes.byref(state)), "sail_server_poll")
        return state.value

    def cancel(self, job_id: int) -> None:
        _check(lib().sail_server_cancel(self._h, int(job_id)), "sail_server_cancel")

    def stats(self) -> dict:
        st = ServerStatsC()
        _check(lib().sail_server_get_stats(self._h, ctypes.byref(st)), "sail_server_get_stats")
        return {k: getattr(st, k) for k, _ in ServerStatsC._fields_}

    def clock(self) -> float:
        return float(lib().sail_server_clock(self._h))
