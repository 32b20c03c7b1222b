"""Python binding of libsmx, the MI355X (gfx950) HIP library for the
superiorized simultaneous band+box projection method.

This module only marshals arguments into the C ABI of ``include/smx.h``:
torch supplies device memory and the stream, every step of the method runs in
the library's HIP kernels.  There is no fallback: if ``libsmx.so`` is missing or
cannot be loaded, importing the binding's entry points raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsmx.so")

STORE = {"f32": 0, "bf16": 1, "f16": 2}
OBJ_NONE, OBJ_SQNORM, OBJ_TV2D, OBJ_LINEAR, OBJ_L1 = 0, 1, 2, 3, 4
BASIC_SIMULT, BASIC_DROP, BASIC_CQ, BASIC_EL, BASIC_EMR = 0, 1, 2, 3, 4
STOP_NONE, STOP_PROX, STOP_DPROX, STOP_MAXIT, STOP_VAR, STOP_SM = 0, 1, 2, 3, 4, 5
DVC_MAX, DVC_MIN = 0, 1  # dose-volume constraints: D_V <= dose, D_V >= dose
RUN_PERTURB, RUN_GRAPH = 1, 2

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENUMERIC = 0, -1, -2, -3, -4, -5
_CODE_NAMES = {EINVAL: "EINVAL", ENOMEM: "ENOMEM", EDEVICE: "EDEVICE", ESTATE: "ESTATE", ENUMERIC: "ENUMERIC"}

# entry points declared in include/smx.h
EXPORTS = [
    "smx_version",
    "smx_last_error",
    "smx_read_rate_probe",
    "smx_operator_create",
    "smx_operator_create_image",
    "smx_operator_destroy",
    "smx_operator_release_panels",
    "smx_operator_footprint",
    "smx_footprint",
    "smx_problem_create",
    "smx_problem_destroy",
    "smx_create",
    "smx_set_stream",
    "smx_set_x",
    "smx_get_x",
    "smx_run",
    "smx_sync",
    "smx_query",
    "smx_get_history",
    "smx_get_state",
    "smx_set_state",
    "smx_problem_dims",
    "smx_set_timing",
    "smx_get_timing",
    "smx_autotune",
    "smx_describe",
    "smx_set_fused",
    "smx_set_fused_shape",
    "smx_set_phase_form",
    "smx_stop_status",
    "smx_slot_load",
    "smx_slot_load_noalloc",
    "smx_slot_disable",
    "smx_slot_status",
    "smx_slot_get_x",
]


STEP_POWER, STEP_ADAPTIVE = 0, 1  # smx_problem_desc.step_rule
PHASE_AUTO, PHASE_ONE_LAUNCH, PHASE_BATCHES, PHASE_CLOSED_FORM = 0, 1, 2, 3  # smx_set_phase_form


class SmxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{_CODE_NAMES.get(code, code)}: {msg}")
        self.code = code


class Csr(C.Structure):
    _fields_ = [
        ("m", C.c_int64),
        ("n", C.c_int64),
        ("nnz", C.c_int64),
        ("row_ptr", C.c_void_p),
        ("col_idx", C.c_void_p),
        ("val", C.c_void_p),
        ("on_device", C.c_int32),
    ]


class DvcC(C.Structure):
    _fields_ = [
        ("row_begin", C.c_int64),
        ("row_end", C.c_int64),
        ("sense", C.c_int32),
        ("reserved", C.c_int32),
        ("fraction", C.c_double),
        ("dose", C.c_double),
    ]


class ProblemDesc(C.Structure):
    _fields_ = [
        ("B", C.c_int32),
        ("lower", C.c_void_p),
        ("upper", C.c_void_p),
        ("weights", C.c_void_p),
        ("box_lo", C.c_void_p),
        ("box_hi", C.c_void_p),
        ("lam", C.c_double),
        ("obj_kind", C.c_int32),
        ("tv_rows", C.c_int32),
        ("tv_cols", C.c_int32),
        ("tv_eps", C.c_double),
        ("linear_c", C.c_void_p),
        ("gamma", C.c_double),
        ("alpha", C.c_double),
        ("n_red", C.c_int32),
        ("restart_every", C.c_int32),
        ("max_trials", C.c_int32),
        ("refine_iters", C.c_int32),
        ("history_cap", C.c_int32),
        ("on_device", C.c_int32),
        ("basic", C.c_int32),
        ("stop_on", C.c_int32),
        ("stop_n", C.c_int32),
        ("stop_max_iters", C.c_int64),
        ("stop_prox", C.c_double),
        ("stop_dprox", C.c_double),
        ("stop_dobj", C.c_double),
        ("stop_var", C.c_double),
        ("n_dvc", C.c_int32),
        ("reserved_dvc", C.c_int32),
        ("dvc", C.POINTER(DvcC)),
        ("step_rule", C.c_int32),
        ("reserved_step", C.c_int32),
    ]


class SliceStateC(C.Structure):
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
        ("reserved", C.c_int32),
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

    def as_dict(self) -> dict:
        """Fields as Python numbers (NaN as None, so equal states compare equal)."""
        out = {}
        for f, t in self._fields_:
            v = getattr(self, f)
            out[f] = (None if v != v else float(v)) if t is C.c_double else int(v)
        return out


_lib = None


def lib() -> C.CDLL:
    """The loaded libsmx.so; raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"libsmx.so not found at {LIB_PATH}: build it with __graft_entry__.build()")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, dbl = C.c_void_p, C.c_int32, C.c_int64, C.c_double
    L.smx_version.argtypes = [C.POINTER(C.c_int), C.POINTER(C.c_int)]
    L.smx_last_error.restype = C.c_char_p
    L.smx_operator_create.argtypes = [C.POINTER(Csr), i32, i32, vp, C.POINTER(vp)]
    L.smx_operator_create_image.argtypes = [C.POINTER(Csr), i32, i32, i32, i32, vp, C.POINTER(vp)]
    L.smx_operator_destroy.argtypes = [vp]
    L.smx_operator_release_panels.argtypes = [vp]
    L.smx_read_rate_probe.argtypes = [vp, C.c_size_t, vp, i32, vp]
    L.smx_operator_footprint.argtypes = [i64, i64, i64, i32, i32, C.POINTER(C.c_size_t)]
    L.smx_footprint.argtypes = [i64, i64, i64, i32, i32, i32, i32, C.POINTER(ProblemDesc), C.POINTER(C.c_size_t),
                                C.POINTER(C.c_size_t)]
    L.smx_problem_create.argtypes = [vp, C.POINTER(ProblemDesc), vp, C.POINTER(vp)]
    L.smx_problem_destroy.argtypes = [vp]
    L.smx_create.argtypes = [C.POINTER(Csr), i32, C.POINTER(ProblemDesc), vp, C.POINTER(vp)]
    L.smx_set_stream.argtypes = [vp, vp]
    L.smx_set_x.argtypes = [vp, vp, i32]
    L.smx_get_x.argtypes = [vp, vp, i32]
    L.smx_run.argtypes = [vp, i32, C.c_uint32]
    L.smx_sync.argtypes = [vp]
    L.smx_query.argtypes = [vp, vp, vp]
    L.smx_get_history.argtypes = [vp, vp, vp, vp, vp, vp, i32, C.POINTER(i32)]
    L.smx_get_state.argtypes = [vp, vp, vp]
    L.smx_set_state.argtypes = [vp, vp, vp]
    L.smx_problem_dims.argtypes = [vp, C.POINTER(i64), C.POINTER(i64), C.POINTER(i64), C.POINTER(i32)]
    L.smx_set_timing.argtypes = [vp, i32]
    L.smx_get_timing.argtypes = [vp, C.POINTER(dbl), C.POINTER(dbl), C.POINTER(i64)]
    L.smx_autotune.argtypes = [vp, i32]
    L.smx_slot_load.argtypes = [vp, i32, vp, vp, vp, i32, i64]
    L.smx_slot_load_noalloc.argtypes = [vp, i32, vp, vp, vp, i32, i64]
    L.smx_slot_disable.argtypes = [vp, i32]
    L.smx_slot_status.argtypes = [vp, vp, vp]
    L.smx_slot_get_x.argtypes = [vp, i32, vp, i32]
    L.smx_describe.argtypes = [vp, C.c_char_p, C.c_size_t, C.POINTER(C.c_size_t)]
    L.smx_set_fused.argtypes = [vp, i32]
    L.smx_set_fused_shape.argtypes = [vp, i32, i32, i32, i32]
    L.smx_set_phase_form.argtypes = [vp, i32]
    L.smx_stop_status.argtypes = [vp, vp]
    for name in EXPORTS:
        if name != "smx_last_error":
            getattr(L, name).restype = C.c_int
    _lib = L
    return L


def check(rc: int) -> None:
    if rc != OK:
        raise SmxError(rc, lib().smx_last_error().decode(errors="replace"))


def version() -> tuple:
    a, b = C.c_int(), C.c_int()
    check(lib().smx_version(C.byref(a), C.byref(b)))
    return a.value, b.value


def _stream_ptr(stream) -> Optional[int]:
    import torch

    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream or None


def _dev(a, dtype, device):
    """A contiguous device tensor holding `a` (numpy array or tensor)."""
    import torch

    if a is None:
        return None
    t = a if isinstance(a, torch.Tensor) else torch.from_numpy(np.ascontiguousarray(a))
    return t.to(device=device, dtype=dtype).contiguous()


def _ptr(t) -> Optional[int]:
    return None if t is None else t.data_ptr()


class Operator:
    """A on the device: row-aligned CSR, column-major copy, row norms and an
    optional reduced-precision value copy (``storage`` in f32 / bf16 / f16)."""

    def __init__(self, m, n, row_ptr, col_idx, val, storage: str = "f32", keep_f32: bool = True,
                 device="cuda", stream=None, image=None):
        """image = (rows, cols): the unknowns are the pixels of that image
        (row-major), which adds the tiled column layout for A^T."""
        import torch

        self.m, self.n = int(m), int(n)
        self.storage = storage
        rp = _dev(row_ptr, torch.int32, device)
        ci = _dev(col_idx, torch.int32, device)
        va = _dev(val, torch.float32, device)
        self.nnz = int(ci.numel())
        csr = Csr(self.m, self.n, self.nnz, _ptr(rp), _ptr(ci), _ptr(va), 1)
        h = C.c_void_p()
        if image is None:
            check(lib().smx_operator_create(C.byref(csr), STORE[storage], 1 if keep_f32 else 0,
                                            _stream_ptr(stream), C.byref(h)))
        else:
            check(lib().smx_operator_create_image(C.byref(csr), STORE[storage], 1 if keep_f32 else 0,
                                                  int(image[0]), int(image[1]), _stream_ptr(stream), C.byref(h)))
        self.handle = h

    def release_panels(self):
        """Free the row-panel layout of the column copy (smx_operator_release_panels):
        for operators whose problems are multi-slice or will not use that pass."""
        check(lib().smx_operator_release_panels(self.handle))

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            check(lib().smx_operator_destroy(self.handle))
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def read_rate_probe(buf, partials, grid: int, stream=None) -> None:
    """One read-only pass over the device tensor buf (smx_read_rate_probe);
    partials: a float32 device tensor of at least grid entries."""
    import torch

    assert buf.is_cuda and partials.is_cuda and partials.dtype == torch.float32 and partials.numel() >= grid
    check(lib().smx_read_rate_probe(_ptr(buf), buf.numel() * buf.element_size(), _ptr(partials), int(grid),
                                    _stream_ptr(stream)))


def footprint(m, n, nnz, storage="f32", keep_f32=True) -> int:
    b = C.c_size_t()
    check(lib().smx_operator_footprint(int(m), int(n), int(nnz), STORE[storage], 1 if keep_f32 else 0, C.byref(b)))
    return int(b.value)


def _desc(B, lower, upper, weights, box_lo, box_hi, linear_c, lam=1.0, obj=OBJ_NONE, tv_rows=0, tv_cols=0,
          tv_eps=0.0, gamma=1.0, alpha=0.99, n_red=1, restart_every=0, max_trials=100, refine_iters=-1,
          history_cap=0, basic=0, stop=None, dvc=None, step_rule=0):
    """The problem descriptor (device pointers or None for the arrays) and the
    dose-volume table it points to (kept alive by the caller)."""
    d = ProblemDesc(
        B=int(B), lower=lower, upper=upper, weights=weights, box_lo=box_lo, box_hi=box_hi, lam=float(lam),
        obj_kind=int(obj), tv_rows=int(tv_rows), tv_cols=int(tv_cols), tv_eps=float(tv_eps), linear_c=linear_c,
        gamma=float(gamma), alpha=float(alpha), n_red=int(n_red), restart_every=int(restart_every),
        max_trials=int(max_trials), refine_iters=int(refine_iters), history_cap=int(history_cap), on_device=1,
        basic=int(basic), step_rule=int(step_rule),
    )
    if stop is not None:  # stopping rules: prox, dprox, n, max_iters, dobj, var
        d.stop_on = 1
        d.stop_n = int(stop.get("n", 5))
        d.stop_max_iters = int(stop.get("max_iters", 0))
        d.stop_prox = float(stop.get("prox", 1e-6))
        d.stop_dprox = float(stop.get("dprox", 1e-8))
        d.stop_dobj = float(stop.get("dobj", 1e-6))
        d.stop_var = float(stop.get("var", 0.0))
    tab = None
    if dvc:
        tab = (DvcC * len(dvc))()
        for i, g in enumerate(dvc):
            tab[i] = DvcC(row_begin=int(g["row_begin"]), row_end=int(g["row_end"]), sense=int(g["sense"]),
                          fraction=float(g["fraction"]), dose=float(g["dose"]))
        d.n_dvc = len(dvc)
        d.dvc = C.cast(tab, C.POINTER(DvcC))
    return d, tab


def problem_footprint(m, n, nnz, storage="f32", keep_f32=True, B=1, image=None, **params) -> tuple:
    """(operator bytes, problem bytes) the library would allocate for an
    operator of this shape (image = (rows, cols): an image operator) and a
    problem with these Problem keyword arguments (bands and other arrays are
    not needed: only sizes count), on the current device, without allocating
    anything."""
    keys = ("lam", "obj", "tv_rows", "tv_cols", "tv_eps", "gamma", "alpha", "n_red", "restart_every", "max_trials",
            "refine_iters", "history_cap", "basic", "stop", "dvc", "step_rule")
    d, tab = _desc(B, None, None, None, None, None, None, **{k: v for k, v in params.items() if k in keys})
    ob, pb = C.c_size_t(), C.c_size_t()
    ir, ic = (0, 0) if image is None else (int(image[0]), int(image[1]))
    check(lib().smx_footprint(int(m), int(n), int(nnz), STORE[storage], 1 if keep_f32 else 0, ir, ic, C.byref(d),
                              C.byref(ob), C.byref(pb)))
    return int(ob.value), int(pb.value)


class Problem:
    """Band+box problem with B slices on an :class:`Operator`."""

    def __init__(self, op: Operator, lower, upper, box_lo=None, box_hi=None, weights=None, lam=1.0,
                 obj=OBJ_NONE, tv_rows=0, tv_cols=0, tv_eps=0.0, linear_c=None, gamma=1.0, alpha=0.99,
                 n_red=1, restart_every=0, max_trials=100, refine_iters=-1, history_cap=0, B=None,
                 device="cuda", stream=None, basic=0, stop=None, dvc=None, step_rule=0):
        """dvc: dose-volume constraints, dicts with row_begin, row_end, sense
        (DVC_MAX / DVC_MIN), fraction and dose; their row blocks consecutive."""
        import torch

        self.op = op
        self.device = device
        lower = np.asarray(lower, np.float32) if not isinstance(lower, torch.Tensor) else lower
        if B is None:
            B = 1 if lower.ndim == 1 else int(lower.shape[1])
        self.B = int(B)
        self.m, self.n = op.m, op.n
        t_lo = _dev(lower, torch.float32, device).reshape(-1)
        t_up = _dev(upper, torch.float32, device).reshape(-1)
        t_w = _dev(weights, torch.float64, device)
        t_blo = _dev(box_lo, torch.float32, device)
        t_bhi = _dev(box_hi, torch.float32, device)
        t_c = _dev(linear_c, torch.float32, device)
        d, self._dvc_tab = _desc(self.B, _ptr(t_lo), _ptr(t_up), _ptr(t_w), _ptr(t_blo), _ptr(t_bhi), _ptr(t_c),
                                 lam=lam, obj=obj, tv_rows=tv_rows, tv_cols=tv_cols, tv_eps=tv_eps, gamma=gamma,
                                 alpha=alpha, n_red=n_red, restart_every=restart_every, max_trials=max_trials,
                                 refine_iters=refine_iters, history_cap=history_cap, basic=basic, stop=stop, dvc=dvc,
                                 step_rule=step_rule)
        self.history_cap = int(history_cap)
        self.obj = int(obj)
        h = C.c_void_p()
        check(lib().smx_problem_create(op.handle, C.byref(d), _stream_ptr(stream), C.byref(h)))
        self.handle = h

    # -- iterate -----------------------------------------------------------
    def set_x(self, x):
        import torch

        t = _dev(x, torch.float32, self.device).reshape(-1)
        assert t.numel() == self.n * self.B
        check(lib().smx_set_x(self.handle, _ptr(t), 1))
        torch.cuda.current_stream().synchronize()

    def get_x(self):
        """Iterate as a device tensor of shape [n, B]."""
        import torch

        out = torch.empty(self.n * self.B, dtype=torch.float32, device=self.device)
        check(lib().smx_get_x(self.handle, _ptr(out), 1))
        return out.reshape(self.n, self.B)

    # -- iteration ---------------------------------------------------------
    def run(self, K: int, perturb: bool = True, graph: bool = False):
        flags = (RUN_PERTURB if perturb else 0) | (RUN_GRAPH if graph else 0)
        check(lib().smx_run(self.handle, int(K), flags))

    def sync(self):
        check(lib().smx_sync(self.handle))

    def set_stream(self, stream):
        check(lib().smx_set_stream(self.handle, _stream_ptr(stream)))

    def query(self):
        """(proximity[B], objective[B]) at the current iterate, float64."""
        p = np.zeros(self.B)
        f = np.zeros(self.B)
        check(lib().smx_query(self.handle, p.ctypes.data, f.ctypes.data))
        return p, f

    def history(self):
        cap = max(self.history_cap, 0)
        shape = (cap, self.B)
        prox = np.zeros(shape)
        fs = np.zeros(shape)
        fe = np.zeros(shape)
        tr = np.zeros(shape, np.int32)
        ac = np.zeros(shape, np.int32)
        n = C.c_int32()
        check(lib().smx_get_history(self.handle, prox.ctypes.data, fs.ctypes.data, fe.ctypes.data, tr.ctypes.data,
                                    ac.ctypes.data, cap, C.byref(n)))
        k = n.value
        return dict(prox=prox[:k], f_start=fs[:k], f_end=fe[:k], trials=tr[:k], accepts=ac[:k])

    def get_state(self):
        st = (SliceStateC * self.B)()
        x = np.zeros(self.n * self.B, np.float32)
        check(lib().smx_get_state(self.handle, C.cast(st, C.c_void_p), x.ctypes.data))
        return [s.as_dict() for s in st], x.reshape(self.n, self.B)

    def set_state(self, states, x):
        st = (SliceStateC * self.B)()
        for i, s in enumerate(states):
            st[i].p_last = st[i].f_last = st[i].f_ref = float("nan")
            for k, v in s.items():
                t = dict(SliceStateC._fields_)[k]
                setattr(st[i], k, (float("nan") if v is None else float(v)) if t is C.c_double else int(v))
        xx = np.ascontiguousarray(np.asarray(x, np.float32).reshape(-1))
        check(lib().smx_set_state(self.handle, C.cast(st, C.c_void_p), xx.ctypes.data))

    def reset(self, x0):
        """Iteration state back to k = ell = restarts = 0 and the iterate to x0."""
        zero = dict(k=0, ell=0, restarts=0, trials=0, accepts=0, cap_hits=0)
        self.set_state([zero] * self.B, np.asarray(x0, np.float32).reshape(self.n, self.B))

    def autotune(self, reps: int = 10) -> dict:
        """Pick the fastest launch shapes of both passes on this operator."""
        check(lib().smx_autotune(self.handle, int(reps)))
        return self.describe()

    def describe(self) -> dict:
        import json

        need = C.c_size_t()
        check(lib().smx_describe(self.handle, None, 0, C.byref(need)))
        buf = C.create_string_buffer(need.value)
        check(lib().smx_describe(self.handle, buf, need.value, None))
        return json.loads(buf.value.decode())

    # -- slots (serving) ---------------------------------------------------
    def slot_load(self, slot: int, lower, upper, x0, budget: int):
        """Load one slot's bands and starting point (host arrays, copied in order
        on the problem's stream); the slot then runs `budget` iterations."""
        lo = np.ascontiguousarray(np.asarray(lower, np.float32).reshape(-1))
        up = np.ascontiguousarray(np.asarray(upper, np.float32).reshape(-1))
        xx = np.ascontiguousarray(np.asarray(x0, np.float32).reshape(-1))
        assert lo.size == self.m and up.size == self.m and xx.size == self.n
        check(lib().smx_slot_load(self.handle, int(slot), lo.ctypes.data, up.ctypes.data, xx.ctypes.data, 0,
                                  int(budget)))

    def slot_load_noalloc(self, slot: int, lower, upper, x0, budget: int):
        """slot_load through the entry point that allocates nothing (its
        staging lives in the library's fixed device scratch).  Device tensors
        are passed as device pointers, anything else as host arrays."""
        import torch

        arrs = [lower, upper, x0]
        if all(isinstance(a, torch.Tensor) and a.is_cuda for a in arrs):
            ts = [a.to(torch.float32).contiguous().reshape(-1) for a in arrs]
            assert ts[0].numel() == self.m and ts[1].numel() == self.m and ts[2].numel() == self.n
            check(lib().smx_slot_load_noalloc(self.handle, int(slot), _ptr(ts[0]), _ptr(ts[1]), _ptr(ts[2]), 1,
                                              int(budget)))
            return
        lo, up, xx = (np.ascontiguousarray(np.asarray(a, np.float32).reshape(-1)) for a in arrs)
        assert lo.size == self.m and up.size == self.m and xx.size == self.n
        check(lib().smx_slot_load_noalloc(self.handle, int(slot), lo.ctypes.data, up.ctypes.data, xx.ctypes.data, 0,
                                          int(budget)))

    def slot_disable(self, slot: int):
        check(lib().smx_slot_disable(self.handle, int(slot)))

    def slot_status(self):
        k = np.zeros(self.B, np.int64)
        live = np.zeros(self.B, np.int32)
        check(lib().smx_slot_status(self.handle, k.ctypes.data, live.ctypes.data))
        return k, live

    def slot_x_host(self, slot: int) -> np.ndarray:
        """Slot iterate copied to the host [n] (waits for the problem's stream)."""
        out = np.empty(self.n, np.float32)
        check(lib().smx_slot_get_x(self.handle, int(slot), out.ctypes.data, 0))
        return out

    def slot_x(self, slot: int):
        """Slot iterate as a device tensor [n]."""
        import torch

        out = torch.empty(self.n, dtype=torch.float32, device=self.device)
        check(lib().smx_slot_get_x(self.handle, int(slot), _ptr(out), 1))
        return out

    def set_fused(self, on: bool):
        """Fused single pass for one-slice problems where it is available (on),
        or always the two bitwise-reproducible passes (off)."""
        check(lib().smx_set_fused(self.handle, 1 if on else 0))

    def set_phase_form(self, form: int):
        """Perturbation phase in one launch per slice (PHASE_ONE_LAUNCH), as a
        chain of trial-batch launches (PHASE_BATCHES), with the linear
        objective's trials in closed form (PHASE_CLOSED_FORM), or chosen by
        objective and size (PHASE_AUTO)."""
        check(lib().smx_set_phase_form(self.handle, int(form)))

    def stop_status(self) -> np.ndarray:
        """Why each slice stopped (STOP_*; 0 while it runs)."""
        r = np.zeros(self.B, np.int32)
        check(lib().smx_stop_status(self.handle, r.ctypes.data))
        return r

    def set_fused_shape(self, lpr: int, vec: int, cap: int, z_in_lds: bool = False):
        """Pin the fused pass's launch shape (see smx_set_fused_shape)."""
        check(lib().smx_set_fused_shape(self.handle, int(lpr), int(vec), int(cap), 1 if z_in_lds else 0))

    def fused_in_use(self) -> bool:
        d = self.describe()
        return any(isinstance(v, dict) and isinstance(v.get("fused"), dict) and v["fused"]["in_use"]
                   for v in d.values())

    def set_timing(self, on: bool):
        check(lib().smx_set_timing(self.handle, 1 if on else 0))

    def timing(self):
        a, b, n = C.c_double(), C.c_double(), C.c_int64()
        check(lib().smx_get_timing(self.handle, C.byref(a), C.byref(b), C.byref(n)))
        return a.value, b.value, n.value

    def close(self):
        if getattr(self, "handle", None) and self.handle.value:
            check(lib().smx_problem_destroy(self.handle))
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def workload_kwargs(w, history_cap: int = 0, refine_iters: int = -1) -> dict:
    """Problem keyword arguments of a :class:`workloads.Workload`."""
    return dict(
        lower=w.lower, upper=w.upper, box_lo=w.box_lo, box_hi=w.box_hi, weights=w.weights, lam=w.lam, obj=w.obj,
        tv_rows=w.tv_rows, tv_cols=w.tv_cols, tv_eps=w.tv_eps, linear_c=w.linear_c, gamma=w.gamma, alpha=w.alpha,
        n_red=w.n_red, restart_every=w.restart_every, max_trials=w.max_trials, history_cap=history_cap,
        refine_iters=refine_iters, B=w.B, basic=getattr(w, "basic", 0), stop=getattr(w, "stop", None),
        dvc=getattr(w, "dvc", None), step_rule=getattr(w, "step_rule", 0),
    )


def problem_from_workload(w, storage: str = "f32", history_cap: int = 0, device="cuda", op: Operator = None,
                          refine_iters: int = -1, fused: bool = True, **overrides) -> Problem:
    """Build operator + problem for a :class:`workloads.Workload` (all slices);
    fused=False keeps the two bitwise-reproducible passes."""
    if op is None:
        op = Operator(w.m, w.n, w.row_ptr, w.col_idx, w.val, storage=storage, device=device,
                      image=getattr(w, "image", None))
    kw = workload_kwargs(w, history_cap, refine_iters)
    kw.update(overrides)
    p = Problem(op, device=device, **kw)
    if not fused:
        p.set_fused(False)
    p.set_x(w.x0)
    return p
