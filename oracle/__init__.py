"""FP64 CPU oracle for the superiorized band+box projection method.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline
leg of the benchmark may import this package; the product path (the HIP
library and its Python binding) never does.  The arithmetic lives in
``orc.c`` (plain C, double precision, written from the paper); this module only
marshals arrays through ``ctypes``.  It shares no code with the HIP path.

Inputs come from :mod:`workloads` as float32 arrays and are promoted exactly to
float64 here.  Weights default to 1/m; caller weights are normalised to sum 1,
as the weighted proximity of Section 2.1.1 requires.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass
from typing import Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "orc.c")
_LIB = os.path.join(_HERE, "liborc.so")

OBJ_NONE, OBJ_SQNORM, OBJ_TV2D, OBJ_LINEAR, OBJ_L1 = 0, 1, 2, 3, 4
STOP_PROX, STOP_DPROX, STOP_MAXIT, STOP_VAR, STOP_SM = 1, 2, 3, 4, 5
BASIC_SIMULT, BASIC_DROP, BASIC_CQ, BASIC_EL, BASIC_EMR = 0, 1, 2, 3, 4
BASIC_ART = 5  # sequential projections, one sweep per iteration (the oracle only)
DVC_MAX, DVC_MIN = 0, 1
STEP_POWER, STEP_ADAPTIVE = 0, 1  # perturbation step size: power law, adaptive (Section 2.1.2)


def build(force: bool = True) -> str:
    """Compile ``orc.c`` with gcc into ``liborc.so`` (no HIP involved)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["gcc", "-O2", "-std=c11", "-fopenmp", "-fPIC", "-shared", "-Wall", "-o", tmp, _SRC, "-lm"]
        )
        os.replace(tmp, _LIB)
    return _LIB


class _Dvc(C.Structure):
    _fields_ = [
        ("row_begin", C.c_int64),
        ("row_end", C.c_int64),
        ("sense", C.c_int32),
        ("pad_", C.c_int32),
        ("fraction", C.c_double),
        ("dose", C.c_double),
    ]


class _Problem(C.Structure):
    _fields_ = [
        ("m", C.c_int64),
        ("n", C.c_int64),
        ("row_ptr", C.POINTER(C.c_int64)),
        ("col", C.POINTER(C.c_int32)),
        ("val", C.POINTER(C.c_double)),
        ("lower", C.POINTER(C.c_double)),
        ("upper", C.POINTER(C.c_double)),
        ("w", C.POINTER(C.c_double)),
        ("box_lo", C.POINTER(C.c_double)),
        ("box_hi", C.POINTER(C.c_double)),
        ("lam", C.c_double),
        ("obj", C.c_int32),
        ("tv_rows", C.c_int32),
        ("tv_cols", C.c_int32),
        ("max_trials", C.c_int32),
        ("tv_eps", C.c_double),
        ("lin_c", C.POINTER(C.c_double)),
        ("gamma", C.c_double),
        ("alpha", C.c_double),
        ("n_red", C.c_int32),
        ("restart_every", C.c_int32),
        ("basic", C.c_int32),
        ("col_nnz", C.POINTER(C.c_double)),
        ("stop_on", C.c_int32),
        ("stop_n", C.c_int32),
        ("stop_max", C.c_int32),
        ("stop_prox", C.c_double),
        ("stop_dprox", C.c_double),
        ("stop_dobj", C.c_double),
        ("stop_var", C.c_double),
        ("n_dvc", C.c_int32),
        ("pad_", C.c_int32),
        ("dvc", C.POINTER(_Dvc)),
        ("csc_ptr", C.POINTER(C.c_int64)),
        ("csc_row", C.POINTER(C.c_int32)),
        ("csc_val", C.POINTER(C.c_double)),
        ("step_rule", C.c_int32),
        ("pad2_", C.c_int32),
    ]


class State(C.Structure):
    """Iteration state of Algorithm 1: k, ell, restarts and trial counters."""

    _fields_ = [
        ("k", C.c_int64),
        ("ell", C.c_int64),
        ("restarts", C.c_int64),
        ("trials", C.c_int64),
        ("accepts", C.c_int64),
        ("cap_hits", C.c_int64),
        ("stop_reason", C.c_int32),
        ("dp_run", C.c_int32),
        ("feas_ok", C.c_int32),
        ("pad_", C.c_int32),
        ("p_last", C.c_double),
        ("f_last", C.c_double),
        ("var_n", C.c_double),
        ("var_mean", C.c_double),
        ("var_m2", C.c_double),
        ("f_ref", C.c_double),
    ]

    def __init__(self):
        super().__init__()
        self.p_last = float("nan")
        self.f_last = float("nan")
        self.f_ref = float("nan")

    def copy(self) -> "State":
        s = State()
        C.pointer(s)[0] = self
        return s

    def as_dict(self) -> dict:
        """Fields as Python numbers (NaN as None, so equal states compare equal)."""
        out = {}
        for f, t in self._fields_:
            v = getattr(self, f)
            out[f] = (None if v != v else float(v)) if t is C.c_double else int(v)
        return out


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        L = C.CDLL(_LIB)
        P = C.POINTER(_Problem)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.orc_matvec.argtypes = [P, dp, dp]
        L.orc_matvec_t.argtypes = [P, dp, dp]
        L.orc_row_sqnorms.argtypes = [P, dp]
        L.orc_proximity.argtypes = [P, dp]
        L.orc_proximity.restype = C.c_double
        L.orc_step.argtypes = [P, dp]
        L.orc_step.restype = C.c_double
        L.orc_objective.argtypes = [P, dp]
        L.orc_objective.restype = C.c_double
        L.orc_gradient.argtypes = [P, dp, dp]
        L.orc_run.argtypes = [P, dp, C.c_int64, C.c_int32, C.POINTER(State), dp, dp, dp, ip, ip]
        L.orc_run.restype = C.c_int
        L.orc_prepare.argtypes = [P, dp, dp]
        L.orc_run_prepared.argtypes = [P, dp, dp, dp, C.c_int64, C.c_int32, C.POINTER(State), dp, dp, dp, ip, ip]
        L.orc_run_prepared.restype = C.c_int
        L.orc_build_csc.argtypes = [P, C.POINTER(C.c_int64), ip, dp]
        L.orc_set_threads.argtypes = [C.c_int32]
        L.orc_max_threads.restype = C.c_int32
        L.orc_dvc_boundary.argtypes = [P, dp, dp, dp]
        L.orc_perturb.argtypes = [P, dp, C.POINTER(State)]
        L.orc_perturb.restype = C.c_int
        L.orc_bands_at.argtypes = [P, dp, dp, dp]
        L.orc_dvc_count.argtypes = [C.POINTER(_Dvc)]
        L.orc_dvc_count.restype = C.c_int64
        L.orc_round_bf16.argtypes = [dp, dp, C.c_int64]
        L.orc_round_f16_scaled.argtypes = [dp, dp, C.c_int64]
        L.orc_round_f16_scaled.restype = C.c_double
        _lib = L
    return _lib


def set_threads(n: int) -> None:
    """OpenMP threads of the oracle's parallel loops (results do not depend on it)."""
    lib().orc_set_threads(int(n))


def max_threads() -> int:
    return int(lib().orc_max_threads())


def _dp(a: Optional[np.ndarray]):
    if a is None:
        return None
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a, dtype=np.float64))


@dataclass
class History:
    prox: np.ndarray
    f_start: np.ndarray
    f_end: np.ndarray
    trials: np.ndarray
    accepts: np.ndarray


class Problem:
    """One slice of a band+box problem, all arrays in float64."""

    def __init__(
        self,
        m,
        n,
        row_ptr,
        col_idx,
        val,
        lower,
        upper,
        box_lo=None,
        box_hi=None,
        weights=None,
        lam=1.0,
        obj=OBJ_NONE,
        tv_rows=0,
        tv_cols=0,
        tv_eps=0.0,
        linear_c=None,
        gamma=1.0,
        alpha=0.99,
        n_red=1,
        restart_every=0,
        max_trials=100,
        basic=BASIC_SIMULT,
        col_nnz=None,
        stop=None,
        dvc=None,
        step_rule=STEP_POWER,
    ):
        self.m, self.n = int(m), int(n)
        self.row_ptr = np.ascontiguousarray(np.asarray(row_ptr, dtype=np.int64))
        self.col_idx = np.ascontiguousarray(np.asarray(col_idx, dtype=np.int32))
        self.val = _f64(val)
        self.lower = _f64(lower).reshape(-1)
        self.upper = _f64(upper).reshape(-1)
        self.box_lo = _f64(np.full(self.n, -np.inf) if box_lo is None else box_lo)
        self.box_hi = _f64(np.full(self.n, np.inf) if box_hi is None else box_hi)
        w = np.full(self.m, 1.0 / max(self.m, 1)) if weights is None else _f64(weights)
        self.w = _f64(w / w.sum())
        self.linear_c = None if linear_c is None else _f64(linear_c)
        self.col_nnz = None if col_nnz is None else _f64(col_nnz)
        self.s = _Problem(
            m=self.m,
            n=self.n,
            row_ptr=self.row_ptr.ctypes.data_as(C.POINTER(C.c_int64)),
            col=self.col_idx.ctypes.data_as(C.POINTER(C.c_int32)),
            val=_dp(self.val),
            lower=_dp(self.lower),
            upper=_dp(self.upper),
            w=_dp(self.w),
            box_lo=_dp(self.box_lo),
            box_hi=_dp(self.box_hi),
            lam=float(lam),
            obj=int(obj),
            tv_rows=int(tv_rows),
            tv_cols=int(tv_cols),
            max_trials=int(max_trials),
            tv_eps=float(tv_eps),
            lin_c=_dp(self.linear_c),
            gamma=float(gamma),
            alpha=float(alpha),
            n_red=int(n_red),
            restart_every=int(restart_every),
            basic=int(basic),
            col_nnz=_dp(self.col_nnz),
            step_rule=int(step_rule),
        )
        self.dvc = None
        if dvc:
            self.dvc = (_Dvc * len(dvc))()
            for i, g in enumerate(dvc):
                self.dvc[i] = _Dvc(row_begin=int(g["row_begin"]), row_end=int(g["row_end"]), sense=int(g["sense"]),
                                   fraction=float(g["fraction"]), dose=float(g["dose"]))
            self.s.n_dvc = len(dvc)
            self.s.dvc = C.cast(self.dvc, C.POINTER(_Dvc))
        if stop is not None:
            self.s.stop_on = 1
            self.s.stop_n = int(stop.get("n", 5))
            self.s.stop_max = int(stop.get("max_iters", 0))
            self.s.stop_prox = float(stop.get("prox", 1e-6))
            self.s.stop_dprox = float(stop.get("dprox", 1e-8))
            self.s.stop_dobj = float(stop.get("dobj", 1e-6))
            self.s.stop_var = float(stop.get("var", 0.0))

    # -- setup -----------------------------------------------------------
    def build_csc(self) -> None:
        """The column copy of A for the (then column-parallel) transposed
        product; built once, on first use."""
        if getattr(self, "_csc", None) is not None:
            return
        nnz = int(self.row_ptr[-1])
        cp = np.empty(self.n + 1, np.int64)
        rows = np.empty(max(nnz, 1), np.int32)
        vals = np.empty(max(nnz, 1), np.float64)
        lib().orc_build_csc(C.byref(self.s), cp.ctypes.data_as(C.POINTER(C.c_int64)),
                            rows.ctypes.data_as(C.POINTER(C.c_int32)), _dp(vals))
        self._csc = (cp, rows, vals)
        self.s.csc_ptr = cp.ctypes.data_as(C.POINTER(C.c_int64))
        self.s.csc_row = rows.ctypes.data_as(C.POINTER(C.c_int32))
        self.s.csc_val = _dp(vals)

    def prepare(self) -> None:
        """Everything the iterations reuse: the column copy, the row norms and
        the DROP column factors (done once; run() calls it)."""
        if getattr(self, "_prep", None) is not None:
            return
        self.build_csc()
        q = np.empty(self.m)
        zc = np.empty(self.n)
        lib().orc_prepare(C.byref(self.s), _dp(q), _dp(zc))
        self._prep = (q, zc)

    # -- building blocks -------------------------------------------------
    def matvec(self, x) -> np.ndarray:
        x = _f64(x)
        r = np.empty(self.m)
        lib().orc_matvec(C.byref(self.s), _dp(x), _dp(r))
        return r

    def matvec_t(self, c) -> np.ndarray:
        self.build_csc()
        c = _f64(c)
        y = np.empty(self.n)
        lib().orc_matvec_t(C.byref(self.s), _dp(c), _dp(y))
        return y

    def row_sqnorms(self) -> np.ndarray:
        q = np.empty(self.m)
        lib().orc_row_sqnorms(C.byref(self.s), _dp(q))
        return q

    def proximity(self, x) -> float:
        return float(lib().orc_proximity(C.byref(self.s), _dp(_f64(x))))

    def bands_at(self, x):
        """The bands of every row at x (dose-volume rows: the bands their
        projection sets there)."""
        lo, up = np.empty(self.m), np.empty(self.m)
        lib().orc_bands_at(C.byref(self.s), _dp(_f64(x)), _dp(lo), _dp(up))
        return lo, up

    def dvc_boundary(self, x):
        """(kth, next): each dose-volume constraint's k-th and (k+1)-th
        highest structure values at x (+inf / -inf where k = 0 / k = N)."""
        k = np.empty(max(self.s.n_dvc, 1))
        nx = np.empty(max(self.s.n_dvc, 1))
        lib().orc_dvc_boundary(C.byref(self.s), _dp(_f64(x)), _dp(k), _dp(nx))
        return k[: self.s.n_dvc], nx[: self.s.n_dvc]

    def dvc_count(self, g: int) -> int:
        """k of dose-volume constraint g: floor(V N_S) (MAX) or ceil(V N_S) (MIN)."""
        return int(lib().orc_dvc_count(C.byref(self.dvc[g])))

    def objective(self, x) -> float:
        return float(lib().orc_objective(C.byref(self.s), _dp(_f64(x))))

    def gradient(self, x) -> np.ndarray:
        g = np.empty(self.n)
        lib().orc_gradient(C.byref(self.s), _dp(_f64(x)), _dp(g))
        return g

    def perturb(self, x, state: Optional[State] = None):
        """The perturbation phase alone of the next outer iteration from x:
        returns (z, state after the phase); k and the trial totals are not
        advanced."""
        z = _f64(x).reshape(-1).copy()
        st = State() if state is None else state.copy()
        if lib().orc_perturb(C.byref(self.s), _dp(z), C.byref(st)) != 0:
            raise MemoryError("oracle perturbation failed to allocate")
        return z, st

    def step(self, x):
        """One feasibility step T; returns (T(x), proximity at x)."""
        xx = _f64(x).copy()
        p = lib().orc_step(C.byref(self.s), _dp(xx))
        return xx, float(p)

    # -- Algorithm 1 -----------------------------------------------------
    def run(self, x0, K: int, perturb: bool = True, state: Optional[State] = None):
        """Run K outer iterations; returns (x_K, state, history)."""
        x = _f64(x0).reshape(-1).copy()
        st = State() if state is None else state.copy()
        K = int(K)
        h = History(
            prox=np.empty(K),
            f_start=np.empty(K),
            f_end=np.empty(K),
            trials=np.empty(K, np.int32),
            accepts=np.empty(K, np.int32),
        )
        ip = C.POINTER(C.c_int32)
        self.prepare()
        q, zc = self._prep
        rc = lib().orc_run_prepared(
            C.byref(self.s),
            _dp(q),
            _dp(zc),
            _dp(x),
            K,
            1 if perturb else 0,
            C.byref(st),
            _dp(h.prox),
            _dp(h.f_start),
            _dp(h.f_end),
            h.trials.ctypes.data_as(ip),
            h.accepts.ctypes.data_as(ip),
        )
        if rc != 0:
            raise MemoryError("oracle run failed to allocate")
        return x, st, h


def round_bf16(a) -> np.ndarray:
    a = _f64(a)
    out = np.empty_like(a)
    lib().orc_round_bf16(_dp(a), _dp(out), a.size)
    return out


def round_f16_scaled(a):
    """Returns (rounded values, scale)."""
    a = _f64(a)
    out = np.empty_like(a)
    s = lib().orc_round_f16_scaled(_dp(a), _dp(out), a.size)
    return out, float(s)


def from_workload(w, s: int = 0, value_round: Optional[str] = None) -> Problem:
    """Oracle problem for slice ``s`` of a :class:`workloads.Workload`.

    ``value_round`` in {None, 'bf16', 'f16'} replaces A's values by the
    oracle's own rounding of them (the operator a reduced-precision store holds).
    """
    val = w.val.astype(np.float64)
    # DROP counts the nonzeros of A as given, before any rounding of the values
    col_nnz = np.bincount(np.asarray(w.col_idx)[w.val != 0], minlength=w.n).astype(np.float64)
    if value_round == "bf16":
        val = round_bf16(val)
    elif value_round == "f16":
        val, _ = round_f16_scaled(val)
    elif value_round is not None:
        raise ValueError(value_round)
    return Problem(
        w.m,
        w.n,
        w.row_ptr,
        w.col_idx,
        val,
        w.lower[:, s],
        w.upper[:, s],
        box_lo=w.box_lo,
        box_hi=w.box_hi,
        weights=w.weights,
        lam=w.lam,
        obj=w.obj,
        tv_rows=w.tv_rows,
        tv_cols=w.tv_cols,
        tv_eps=w.tv_eps,
        linear_c=w.linear_c,
        gamma=w.gamma,
        alpha=w.alpha,
        n_red=w.n_red,
        restart_every=w.restart_every,
        max_trials=w.max_trials,
        basic=getattr(w, "basic", BASIC_SIMULT),
        col_nnz=col_nnz,
        stop=getattr(w, "stop", None),
        dvc=getattr(w, "dvc", None),
        step_rule=getattr(w, "step_rule", STEP_POWER),
    )
