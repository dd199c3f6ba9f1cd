"""Plain FP64 CPU oracle for the SAIL annealing method (arXiv:1609.07936).

TEST INFRASTRUCTURE, NOT PRODUCT CODE.  Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import this package.  It wraps ``sail_oracle.c`` (built with ``gcc -O2
-ffp-contract=off``) through ctypes and shares no code with the GPU library.

Sections cited below are those of the paper: Sec. 2.1 spectral model and
kernel, Sec. 2.2 sum-rule preserving moves, Sec. 2.3 index selection,
Sec. 2.5 imprinted branching, Sec. 2.7 amplitude heuristic, Sec. 3 defaults.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "sail_oracle.c")
# SAIL_ORACLE_LIB names another build of the same source (the sanitizer run)
_LIB = os.environ.get("SAIL_ORACLE_LIB") or os.path.join(_HERE, "libsail_oracle.so")
SANITIZE_FLAGS = ["-fsanitize=address,undefined", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer", "-g"]

POINT = 0
BIN_EXACT = 1


def build(force: bool = True, out: str | None = None, sanitize: bool = False) -> str:
    """Compile the oracle with gcc (plain C, OpenMP across walkers only);
    sanitize adds AddressSanitizer and UndefinedBehaviorSanitizer."""
    lib_path = out or _LIB
    if force or not os.path.exists(lib_path):
        tmp = lib_path + ".tmp"
        cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c11",
               "-shared", "-fPIC", *(SANITIZE_FLAGS if sanitize else []), "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, lib_path)
    return lib_path


_lib = None


def lib() -> ctypes.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = ctypes.CDLL(_LIB)
        _declare(_lib)
    return _lib


class AnnealArgs(ctypes.Structure):
    _fields_ = [
        ("n_omega", ctypes.c_int), ("n_tau", ctypes.c_int), ("n_walkers", ctypes.c_int),
        ("omega", ctypes.c_void_p), ("Ft", ctypes.c_void_p), ("w", ctypes.c_void_p), ("K", ctypes.c_void_p),
        ("A", ctypes.c_double), ("B", ctypes.c_double),
        ("T", ctypes.c_void_p), ("n_T", ctypes.c_int), ("chi2_unit", ctypes.c_double),
        ("branch_every", ctypes.c_int), ("resync_every", ctypes.c_int),
        ("branch_fraction", ctypes.c_double), ("imprint_t", ctypes.c_double),
        ("eps0", ctypes.c_double), ("amp_p", ctypes.c_double), ("amp_avg", ctypes.c_double),
        ("amp_m", ctypes.c_int), ("walk_len", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("trace_k0", ctypes.c_int), ("trace_k1", ctypes.c_int),
        ("trace_dchi2", ctypes.c_void_p), ("trace_cond", ctypes.c_void_p),
        ("trace_accept", ctypes.c_void_p), ("replay_accept", ctypes.c_void_p),
        ("band", ctypes.c_double),
        ("max_events", ctypes.c_int),
        ("ev_delta", ctypes.c_void_p), ("ev_pr", ctypes.c_void_p),
        ("ev_z", ctypes.c_void_p), ("ev_status", ctypes.c_void_p), ("ev_m", ctypes.c_void_p),
        ("walker_ids", ctypes.c_void_p),
        ("n_near_ties", ctypes.c_int64), ("n_hard_mismatch", ctypes.c_int64),
        ("n_proposals", ctypes.c_int64), ("n_accepted", ctypes.c_int64),
        ("first_mismatch", ctypes.c_int32 * 3),
        ("trace_p", ctypes.c_void_p), ("trace_s", ctypes.c_void_p),
        ("smooth", ctypes.c_double), ("adaptive", ctypes.c_int),
        ("self_cool", ctypes.c_int), ("boil_blocks", ctypes.c_int), ("cool_blocks", ctypes.c_int),
        ("T_self", ctypes.c_void_p),
        ("ev_gap", ctypes.c_void_p), ("ev_bracket", ctypes.c_void_p), ("ev_robust", ctypes.c_void_p),
        ("replay_m", ctypes.c_void_p), ("replay_m_events", ctypes.c_int),
        ("branch_band", ctypes.c_double),
        ("n_branch_near_ties", ctypes.c_int64), ("n_branch_hard", ctypes.c_int64),
        ("first_branch_mismatch", ctypes.c_int32),
    ]

# Relative perturbation of the residues against which a branching event's
# outcome must be robust (the bar to which two sides' residues agree at an
# event).  An event whose multipliers change under such a perturbation is a
# branching near-tie; at every other event the multipliers must agree exactly.
BRANCH_BAND = 1e-9


def _declare(L: ctypes.CDLL) -> None:
    P = ctypes.c_void_p
    L.or_philox4x32_10.argtypes = [P, P, P]
    L.or_kernel_table.argtypes = [ctypes.c_int, P, ctypes.c_int, P, ctypes.c_int, P]
    L.or_kernel_table.restype = ctypes.c_int
    L.or_forward.argtypes = [P, ctypes.c_int, ctypes.c_int, P, P]
    L.or_chi2.argtypes = [P, P, P, ctypes.c_int]
    L.or_chi2.restype = ctypes.c_double
    L.or_renormalize.argtypes = [P, P, ctypes.c_int, ctypes.c_double, ctypes.c_double]
    L.or_smooth.argtypes = [P, ctypes.c_int, ctypes.c_double]
    L.or_init_spectrum.argtypes = [P, ctypes.c_int, ctypes.c_double, ctypes.c_double, P, P]
    L.or_init_spectrum.restype = ctypes.c_int
    L.or_branch_solve.argtypes = [ctypes.c_int, P, P, ctypes.c_double, P, P, P, P, P, P, P]
    L.or_branch_robust.argtypes = [ctypes.c_int, P, P, ctypes.c_double, ctypes.c_int, P, ctypes.c_double]
    L.or_branch_robust.restype = ctypes.c_int
    L.or_branch_solve.restype = ctypes.c_int
    L.or_branch_pairs.argtypes = [ctypes.c_int, P, P, P]
    L.or_branch_pairs.restype = ctypes.c_int
    L.or_anneal.argtypes = [ctypes.POINTER(AnnealArgs), ctypes.c_int, ctypes.c_int, P, P, P, P]
    L.or_anneal.restype = ctypes.c_int
    L.or_walkers_init.argtypes = [ctypes.POINTER(AnnealArgs), P, P, P, P, P]
    L.or_mean_spectrum.argtypes = [ctypes.c_int, ctypes.c_int, P, P]
    L.or_chi2_hist.argtypes = [ctypes.c_int, P, ctypes.c_int, ctypes.c_double, ctypes.c_double, P]
    L.or_max_threads.restype = ctypes.c_int
    L.or_set_threads.argtypes = [ctypes.c_int]
    L.or_set_threads.restype = None
    L.or_move_deltas.argtypes = [P, ctypes.c_double, ctypes.c_double, ctypes.c_int, ctypes.c_int, ctypes.c_double, P, P]


def _p(a: np.ndarray | None):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


# --------------------------------------------------------------------------
# elementary pieces
# --------------------------------------------------------------------------
def philox4x32_10(ctr, key) -> np.ndarray:
    c = np.ascontiguousarray(ctr, dtype=np.uint32)
    k = np.ascontiguousarray(key, dtype=np.uint32)
    out = np.zeros(4, dtype=np.uint32)
    lib().or_philox4x32_10(_p(c), _p(k), _p(out))
    return out


def kernel_table(mode: int, omega, tau) -> np.ndarray:
    """K[j, i] for bin centre omega_j and time tau_i (Sec. 2.1)."""
    om, ta = _f64(omega), _f64(tau)
    K = np.zeros((om.size, ta.size))
    if lib().or_kernel_table(int(mode), _p(om), om.size, _p(ta), ta.size, _p(K)) != 0:
        raise ValueError("bad grid")
    return K


def forward(K: np.ndarray, a) -> np.ndarray:
    a = _f64(a)
    F = np.zeros(K.shape[1])
    lib().or_forward(_p(np.ascontiguousarray(K)), K.shape[0], K.shape[1], _p(a), _p(F))
    return F


def chi2(F, Ft, w) -> float:
    F, Ft, w = _f64(F), _f64(Ft), _f64(w)
    return float(lib().or_chi2(_p(F), _p(Ft), _p(w), F.size))


def renormalize(a, omega, A: float, B: float) -> np.ndarray:
    a = _f64(a).copy()
    om = _f64(omega)
    lib().or_renormalize(_p(a), _p(om), om.size, float(A), float(B))
    return a


def smooth(a, s: float) -> np.ndarray:
    """The three-point smoothing stencil of Sec. 2.6 with amplitude s."""
    a = _f64(a).copy()
    lib().or_smooth(_p(a), a.size, float(s))
    return a


def init_spectrum(omega, A: float, B: float) -> tuple[np.ndarray, float]:
    om = _f64(omega)
    a = np.zeros(om.size)
    lam = ctypes.c_double(0.0)
    if lib().or_init_spectrum(_p(om), om.size, float(A), float(B), _p(a), ctypes.byref(lam)) != 0:
        raise ValueError("infeasible sum rules: B/A outside the frequency window")
    return a, lam.value


def branch_solve(chi2_values, xi, fraction: float) -> dict:
    c, x = _f64(chi2_values), _f64(xi)
    n = c.size
    m = np.zeros(n, dtype=np.int32)
    delta, pr = ctypes.c_double(), ctypes.c_double()
    z, tie = ctypes.c_int(), ctypes.c_int()
    gap, bracket = ctypes.c_double(), ctypes.c_double()
    st = lib().or_branch_solve(n, _p(c), _p(x), float(fraction), ctypes.byref(delta), ctypes.byref(pr),
                               _p(m), ctypes.byref(z), ctypes.byref(tie), ctypes.byref(gap), ctypes.byref(bracket))
    st_eff = 2 if (st == 0 and tie.value) else st
    robust = lib().or_branch_robust(n, _p(c), _p(x), float(fraction), st_eff,
                                    _p(m if st_eff == 0 else np.ones(n, dtype=np.int32)), BRANCH_BAND)
    return {"status": st, "delta": delta.value, "pr": pr.value, "m": m, "z": z.value, "tie": tie.value,
            "gap": gap.value, "bracket": bracket.value, "robust": bool(robust)}


def branch_robust(chi2_values, xi, fraction: float, status: int, m, eps: float) -> bool:
    """Whether a solve ending with (status, m) keeps that outcome when the
    residues are perturbed by eps relative in four sign patterns."""
    c, x = _f64(chi2_values), _f64(xi)
    mm = np.ascontiguousarray(m, dtype=np.int32)
    return bool(lib().or_branch_robust(c.size, _p(c), _p(x), float(fraction), int(status), _p(mm), float(eps)))


def branch_pairs(m) -> tuple[np.ndarray, np.ndarray]:
    m = np.ascontiguousarray(m, dtype=np.int32)
    tg = np.zeros(m.size, dtype=np.int32)
    dn = np.zeros(m.size, dtype=np.int32)
    npairs = lib().or_branch_pairs(m.size, _p(m), _p(tg), _p(dn))
    if npairs < 0:
        raise ValueError("multipliers do not sum to the population")
    return tg[:npairs].copy(), dn[:npairs].copy()


def chi2_hist(chi2_values, n_bins: int, lo: float, hi: float) -> np.ndarray:
    c = _f64(chi2_values)
    counts = np.zeros(n_bins, dtype=np.uint64)
    lib().or_chi2_hist(c.size, _p(c), int(n_bins), float(lo), float(hi), _p(counts))
    return counts


def move_deltas(omega, A: float, B: float, p: int, s: int, r: float) -> tuple[float, float]:
    """delta_p, delta_s of the sum-rule preserving move (Eqs. update-delta-p/s)."""
    om = _f64(omega)
    dp, ds = ctypes.c_double(), ctypes.c_double()
    lib().or_move_deltas(_p(om), float(A), float(B), int(p), int(s), float(r), ctypes.byref(dp), ctypes.byref(ds))
    return dp.value, ds.value


def max_threads() -> int:
    return int(lib().or_max_threads())


def set_threads(n: int) -> None:
    lib().or_set_threads(int(n))


# --------------------------------------------------------------------------
# problem + anneal runner
# --------------------------------------------------------------------------
@dataclass
class Problem:
    """Inputs of one inversion: bin centres omega (uniform), times tau, data
    Ft with errors sigma (None means the paper's unweighted chi^2), and the
    zeroth/first moments m0 = int S, m1 = int omega S of the spectrum."""
    omega: np.ndarray
    tau: np.ndarray
    Ft: np.ndarray
    sigma: np.ndarray | None
    m0: float
    m1: float
    mode: int = POINT
    K: np.ndarray = field(init=False)
    w: np.ndarray = field(init=False)
    A: float = field(init=False)
    B: float = field(init=False)

    def __post_init__(self):
        self.omega = _f64(self.omega)
        self.tau = _f64(self.tau)
        self.Ft = _f64(self.Ft)
        dw = self.omega[1] - self.omega[0]
        self.K = kernel_table(self.mode, self.omega, self.tau)
        self.w = np.ones(self.tau.size) if self.sigma is None else 1.0 / (_f64(self.sigma) ** 2)
        # Sec. 2.2: int S = d_omega A and int omega S = d_omega B.
        self.A = self.m0 / dw
        self.B = self.m1 / dw


@dataclass
class Schedule:
    """Temperatures T[k] of global sweep k, in units of the starting residue
    (Sec. 3), plus the block and move parameters (Sec. 3 defaults)."""
    T: np.ndarray
    branch_every: int = 100
    resync_every: int = 100
    branch_fraction: float = 0.25
    imprint_t: float = 0.1
    eps0: float = 0.1
    amp_p: float = 1.0
    amp_m: int = 2
    amp_avg: float = 0.1
    walk_len: int = 0
    smooth: float = 0.0
    adaptive: int = 0
    self_cool: int = 0
    boil_blocks: int = 0
    cool_blocks: int = 1


def geometric_schedule(t_hi: float, t_lo: float, n_sweeps: int) -> np.ndarray:
    k = np.arange(n_sweeps, dtype=np.float64)
    if n_sweeps == 1:
        return np.array([t_hi])
    return t_hi * (t_lo / t_hi) ** (k / (n_sweeps - 1))


class Anneal:
    """A walker population advanced by the oracle; state lives in numpy."""

    def __init__(self, prob: Problem, sched: Schedule, n_walkers: int, seed: int, walker_ids=None):
        """walker_ids: optional global numbers of the walkers held here (a
        sample of a larger population; stretches without branching only)."""
        self.prob, self.sched, self.seed = prob, sched, int(seed)
        self.walker_ids = None if walker_ids is None else np.ascontiguousarray(walker_ids, dtype=np.int32)
        self.n = int(n_walkers) if walker_ids is None else int(self.walker_ids.size)
        No, Nt = prob.omega.size, prob.tau.size
        self.a0, self.lam = init_spectrum(prob.omega, prob.A, prob.B)
        self.a = np.zeros((self.n, No))
        self.F = np.zeros((self.n, Nt))
        self.chi2 = np.zeros(self.n)
        self.rate = np.zeros(self.n)
        self._T = _f64(sched.T)
        self.args = AnnealArgs()
        g = self.args
        g.n_omega, g.n_tau, g.n_walkers = No, Nt, self.n
        self._keep = [prob.omega, prob.Ft, prob.w, prob.K, self._T]
        g.omega, g.Ft, g.w, g.K = _p(prob.omega), _p(prob.Ft), _p(prob.w), _p(prob.K)
        g.A, g.B = prob.A, prob.B
        g.T, g.n_T = _p(self._T), self._T.size
        g.branch_every, g.resync_every = sched.branch_every, sched.resync_every
        g.branch_fraction, g.imprint_t = sched.branch_fraction, sched.imprint_t
        g.eps0, g.amp_p, g.amp_m, g.walk_len = sched.eps0, sched.amp_p, sched.amp_m, sched.walk_len
        g.amp_avg = sched.amp_avg
        g.smooth = sched.smooth
        g.adaptive = int(sched.adaptive)
        g.self_cool, g.boil_blocks = int(sched.self_cool), int(sched.boil_blocks)
        g.cool_blocks = int(sched.cool_blocks)
        self.T_self = np.zeros(self._T.size)  # temperatures used under self-cooling (absolute)
        g.T_self = _p(self.T_self)
        g.seed = self.seed
        g.trace_k0 = g.trace_k1 = 0
        g.band = 1e-12
        n_ev = self._T.size // sched.branch_every + 1
        self.ev_delta = np.zeros(n_ev)
        self.ev_pr = np.zeros(n_ev)
        self.ev_z = np.zeros(n_ev, dtype=np.int32)
        self.ev_status = np.full(n_ev, -1, dtype=np.int32)
        self.ev_m = np.zeros((n_ev, self.n), dtype=np.int32)
        self.ev_gap = np.full(n_ev, np.inf)
        self.ev_bracket = np.full(n_ev, np.inf)
        self.ev_robust = np.full(n_ev, -1, dtype=np.int32)
        g.ev_gap, g.ev_bracket, g.ev_robust = _p(self.ev_gap), _p(self.ev_bracket), _p(self.ev_robust)
        g.branch_band = BRANCH_BAND
        g.max_events = n_ev
        g.ev_delta, g.ev_pr, g.ev_z = _p(self.ev_delta), _p(self.ev_pr), _p(self.ev_z)
        g.ev_status, g.ev_m = _p(self.ev_status), _p(self.ev_m)
        g.walker_ids = _p(self.walker_ids)
        lib().or_walkers_init(ctypes.byref(g), _p(self.a0), _p(self.a), _p(self.F), _p(self.chi2),
                              _p(self.rate))
        self.chi2_unit = float(self.chi2[0])  # Sec. 3: the starting residue is the unit of T
        g.chi2_unit = self.chi2_unit

    def run(self, k0: int, k1: int, trace: tuple[int, int] | None = None, replay: np.ndarray | None = None,
            band: float = 1e-12, replay_m: np.ndarray | None = None) -> dict:
        """replay_m: multipliers of events 0.. taken elsewhere ([event][walker]);
        at an event whose outcome is not robust to a relative perturbation
        BRANCH_BAND of the residues they are adopted where they differ (a
        logged branching near-tie), at any other event a difference counts as
        a hard branching mismatch."""
        g = self.args
        No = self.prob.omega.size
        out = {}
        rep_m = None
        if replay_m is not None:
            rep_m = np.ascontiguousarray(replay_m, dtype=np.int32)
            assert rep_m.ndim == 2 and rep_m.shape[1] == self.n
            g.replay_m, g.replay_m_events = _p(rep_m), rep_m.shape[0]
        else:
            g.replay_m, g.replay_m_events = None, 0
        if trace is not None:
            tk0, tk1 = trace
            shape = (self.n, tk1 - tk0, No)
            out["dchi2"] = np.zeros(shape)
            out["cond"] = np.zeros(shape)
            out["accept"] = np.zeros(shape, dtype=np.uint8)
            out["p"] = np.zeros(shape, dtype=np.int32)
            out["s"] = np.zeros(shape, dtype=np.int32)
            g.trace_k0, g.trace_k1 = tk0, tk1
            g.trace_dchi2, g.trace_cond = _p(out["dchi2"]), _p(out["cond"])
            g.trace_accept = _p(out["accept"])
            g.trace_p, g.trace_s = _p(out["p"]), _p(out["s"])
            if replay is not None:
                rep = np.ascontiguousarray(replay, dtype=np.uint8)
                assert rep.shape == shape
                out["_replay"] = rep
                g.replay_accept = _p(rep)
            else:
                g.replay_accept = None
            g.band = band
        else:
            g.trace_k0 = g.trace_k1 = 0
            g.trace_dchi2 = g.trace_cond = g.trace_accept = g.replay_accept = None
            g.trace_p = g.trace_s = None
        g.n_near_ties = g.n_hard_mismatch = g.n_proposals = g.n_accepted = 0
        g.n_branch_near_ties = g.n_branch_hard = 0
        g.first_branch_mismatch = -1
        rc = lib().or_anneal(ctypes.byref(g), int(k0), int(k1), _p(self.a), _p(self.F), _p(self.chi2),
                             _p(self.rate))
        g.replay_m, g.replay_m_events = None, 0
        del rep_m
        if rc == 2:
            raise ValueError("a walker sample cannot cross a branching event")
        if rc != 0:
            raise ValueError("or_anneal rejected its arguments")
        out.update(near_ties=g.n_near_ties, hard_mismatch=g.n_hard_mismatch, proposals=g.n_proposals,
                   accepted=g.n_accepted, first_mismatch=tuple(g.first_mismatch),
                   branch_near_ties=g.n_branch_near_ties, branch_hard=g.n_branch_hard,
                   first_branch_mismatch=g.first_branch_mismatch)
        g.trace_k0 = g.trace_k1 = 0
        g.trace_dchi2 = g.trace_cond = g.trace_accept = g.replay_accept = None
        g.trace_p = g.trace_s = None
        return out

    def mean_spectrum(self) -> np.ndarray:
        out = np.zeros(self.prob.omega.size)
        lib().or_mean_spectrum(self.n, self.prob.omega.size, _p(self.a), _p(out))
        return out


def u01(x) -> np.ndarray:
    """The word-to-uniform map used by both the oracle and its tests."""
    return (np.asarray(x, dtype=np.float64) + 0.5) * 2.0 ** -32


def branch_xi(seed: int, event: int, n_walkers: int) -> np.ndarray:
    """xi_l of branching event e: first word of Philox(l, e, 0, 'BRNC')."""
    key = (seed & 0xFFFFFFFF, seed >> 32)
    return np.array([u01(philox4x32_10((l, event, 0, 0x42524E43), key)[0]) for l in range(n_walkers)])
