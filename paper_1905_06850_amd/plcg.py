"""ctypes binding of libplcg (argument marshalling only).

Each function has the name and arguments of the C entry point in include/plcg.h;
device vectors are passed as integer addresses (for a torch tensor on the GPU,
``t.data_ptr()``) and streams as integer hipStream_t handles (for torch,
``torch.cuda.current_stream().cuda_stream``).  The ``Solver`` class is a small
convenience wrapper over the same calls.  All computation happens in the HIP
library; if it has not been built, importing this module fails.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libplcg.so")

PLCG_OK = 0
PLCG_NOT_READY = 1
PLCG_E_INVALID = -1
PLCG_E_NOMEM = -2
PLCG_E_HIP = -3
PLCG_E_BUSY = -4
PLCG_E_NONFINITE = -5

PLCG_OP_STENCIL2D5 = 1
PLCG_OP_STENCIL3D7 = 2
PLCG_OP_CSR = 3
PLCG_OP_DIAG = 4
PLCG_METHOD_CG = 0
PLCG_METHOD_PLCG = 1
PLCG_PREC_FP64 = 0
PLCG_PREC_FP32_REFINED = 1
PLCG_LAUNCH_AUTO = 0
PLCG_LAUNCH_STREAMING = 1
PLCG_LAUNCH_RESIDENT = 2
PLCG_RESIDENT_MAX = 4800
PLCG_X_AUTO = 0
PLCG_X_EVERY = 1
PLCG_X_PAIRED = 2
LAUNCH_MODES = {"auto": PLCG_LAUNCH_AUTO, "streaming": PLCG_LAUNCH_STREAMING,
                "resident": PLCG_LAUNCH_RESIDENT}
X_UPDATES = {"auto": PLCG_X_AUTO, "every": PLCG_X_EVERY, "paired": PLCG_X_PAIRED}

PLCG_REASON_NONE = 0
PLCG_REASON_CONVERGED = 1
PLCG_REASON_MAXIT = 2
PLCG_REASON_BREAKDOWN_LIMIT = 3
PLCG_REASON_NONFINITE = 4
PLCG_REASON_BREAKDOWN = 5
REASONS = {0: "none", 1: "converged", 2: "maxit", 3: "breakdown_limit", 4: "nonfinite",
           5: "breakdown"}


class plcg_operator_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("diag", ctypes.c_void_p), ("nnz", ctypes.c_int64),
                ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p),
                ("vals", ctypes.c_void_p), ("jacobi", ctypes.c_int32),
                ("cx", ctypes.c_void_p), ("cy", ctypes.c_void_p), ("cz", ctypes.c_void_p)]


class plcg_config(ctypes.Structure):
    _fields_ = [("method", ctypes.c_int32), ("l", ctypes.c_int32),
                ("lambda_min", ctypes.c_double), ("lambda_max", ctypes.c_double),
                ("shifts", ctypes.POINTER(ctypes.c_double)),
                ("check_every", ctypes.c_int32), ("max_restarts", ctypes.c_int32),
                ("history_cap", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("inner_tol", ctypes.c_double), ("launch_mode", ctypes.c_int32),
                ("x_update", ctypes.c_int32)]


class plcg_result(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("spmvs", ctypes.c_int32),
                ("restarts", ctypes.c_int32), ("reason", ctypes.c_int32),
                ("rnorm0", ctypes.c_double), ("rec_relres", ctypes.c_double),
                ("true_relres", ctypes.c_double), ("seconds", ctypes.c_double),
                ("sweep_ms", ctypes.c_double), ("sweeps", ctypes.c_int64),
                ("outer", ctypes.c_int32), ("host_waits", ctypes.c_int32),
                ("launch_mode", ctypes.c_int32), ("x_update_every", ctypes.c_int32)]

    def as_dict(self):
        d = {name: getattr(self, name) for name, _ in self._fields_}
        d["reason_name"] = REASONS.get(self.reason, str(self.reason))
        return d


class plcg_batch_config(ctypes.Structure):
    _fields_ = [("l", ctypes.c_int32), ("lambda_min", ctypes.c_double),
                ("lambda_max", ctypes.c_double), ("max_slots", ctypes.c_int32),
                ("arena_bytes", ctypes.c_int64), ("chunks_per_block", ctypes.c_int32),
                ("max_restarts", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("precision", ctypes.c_int32), ("inner_tol", ctypes.c_double)]


class plcg_system_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("nx", ctypes.c_int32), ("ny", ctypes.c_int32),
                ("nz", ctypes.c_int32), ("cx", ctypes.POINTER(ctypes.c_double)),
                ("cy", ctypes.POINTER(ctypes.c_double)), ("cz", ctypes.POINTER(ctypes.c_double))]


class plcg_request(ctypes.Structure):
    _fields_ = [("arrival_s", ctypes.c_double), ("system", ctypes.c_int32),
                ("maxit", ctypes.c_int32), ("tol", ctypes.c_double), ("x", ctypes.c_void_p)]


class plcg_request_outcome(ctypes.Structure):
    _fields_ = [("admit_s", ctypes.c_double), ("finish_s", ctypes.c_double),
                ("result", plcg_result)]


if not os.path.exists(LIB_PATH):
    raise ImportError(f"libplcg.so is not built ({LIB_PATH}); run __graft_entry__.build()")
_lib = ctypes.CDLL(LIB_PATH)

_h = ctypes.c_void_p
_dp = ctypes.c_void_p       # device pointer as an address
_st = ctypes.c_int32

SYMBOLS = {
    "plcg_create": (_st, [ctypes.POINTER(plcg_operator_desc), ctypes.POINTER(plcg_config),
                          ctypes.POINTER(_h)]),
    "plcg_solve": (_st, [_h, _dp, _dp, ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                         ctypes.POINTER(plcg_result)]),
    "plcg_submit": (_st, [_h, _dp, _dp, ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                          ctypes.POINTER(ctypes.c_uint64)]),
    "plcg_poll": (_st, [_h, ctypes.c_uint64, ctypes.POINTER(plcg_result)]),
    "plcg_destroy": (_st, [_h]),
    "plcg_last_error": (ctypes.c_char_p, []),
    "plcg_apply": (_st, [_h, _dp, _dp, ctypes.c_void_p]),
    "plcg_size": (ctypes.c_int64, [_h]),
    "plcg_get_shifts": (_st, [_h, ctypes.POINTER(ctypes.c_double)]),
    "plcg_get_history": (_st, [_h, ctypes.POINTER(ctypes.c_double), ctypes.c_int32,
                               ctypes.POINTER(ctypes.c_int32)]),
    "plcg_set_timing": (_st, [_h, ctypes.c_int32]),
    "plcg_copy": (_st, [_dp, _dp, ctypes.c_int64, ctypes.c_void_p]),
    "plcg_version": (ctypes.c_int32, []),
    "plcg_solve_noalloc": (_st, [ctypes.POINTER(plcg_operator_desc), ctypes.POINTER(plcg_config),
                                 _dp, _dp, ctypes.c_double, ctypes.c_int32, ctypes.c_void_p,
                                 ctypes.POINTER(plcg_result)]),
    "plcg_resident_supported": (ctypes.c_int32, [ctypes.c_int32, ctypes.c_int64, ctypes.c_int32,
                                                 ctypes.c_int32]),
    "plcg_batch_create": (_st, [ctypes.POINTER(plcg_batch_config), ctypes.POINTER(_h)]),
    "plcg_batch_footprint": (ctypes.c_int64, [_h, ctypes.POINTER(plcg_system_desc)]),
    "plcg_batch_add": (_st, [_h, ctypes.POINTER(plcg_system_desc), _dp, _dp, ctypes.c_double,
                             ctypes.c_int32, ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "plcg_batch_step": (_st, [_h, ctypes.c_int32, ctypes.c_void_p]),
    "plcg_batch_poll": (_st, [_h, ctypes.c_uint64, ctypes.POINTER(plcg_result)]),
    "plcg_batch_active": (ctypes.c_int32, [_h]),
    "plcg_batch_grid": (ctypes.c_int32, [_h]),
    "plcg_batch_chunks_per_block": (ctypes.c_int32, [_h]),
    "plcg_batch_get_schedule": (_st, [_h, ctypes.POINTER(ctypes.c_int32)]),
    "plcg_batch_set_schedule": (_st, [_h, ctypes.POINTER(ctypes.c_int32)]),
    "plcg_batch_autotune": (_st, [_h, ctypes.c_int32, ctypes.c_void_p]),
    "plcg_batch_destroy": (_st, [_h]),
    "plcg_batch_register": (_st, [_h, ctypes.POINTER(plcg_system_desc), ctypes.c_void_p,
                                  ctypes.POINTER(ctypes.c_int32)]),
    "plcg_batch_request_footprint": (ctypes.c_int64, [_h, ctypes.c_int32, ctypes.c_int32]),
    "plcg_batch_add_op": (_st, [_h, ctypes.c_int32, _dp, _dp, ctypes.c_double, ctypes.c_int32,
                                ctypes.c_void_p, ctypes.POINTER(ctypes.c_uint64)]),
    "plcg_serve": (_st, [_h, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_void_p),
                         ctypes.c_int32, ctypes.POINTER(plcg_request), ctypes.c_int32,
                         ctypes.c_int32, ctypes.c_double, ctypes.c_void_p,
                         ctypes.POINTER(plcg_request_outcome)]),
}
for _name, (_res, _args) in SYMBOLS.items():
    _fn = getattr(_lib, _name)
    _fn.restype = _res
    _fn.argtypes = _args

plcg_create = _lib.plcg_create
plcg_solve = _lib.plcg_solve
plcg_submit = _lib.plcg_submit
plcg_poll = _lib.plcg_poll
plcg_destroy = _lib.plcg_destroy
plcg_last_error = _lib.plcg_last_error
plcg_apply = _lib.plcg_apply
plcg_size = _lib.plcg_size
plcg_get_shifts = _lib.plcg_get_shifts
plcg_get_history = _lib.plcg_get_history
plcg_set_timing = _lib.plcg_set_timing
plcg_copy = _lib.plcg_copy
plcg_version = _lib.plcg_version
plcg_solve_noalloc = _lib.plcg_solve_noalloc
PLCG_NOALLOC_BYTES = 64 << 20
plcg_resident_supported = _lib.plcg_resident_supported
plcg_batch_create = _lib.plcg_batch_create
plcg_batch_footprint = _lib.plcg_batch_footprint
plcg_batch_add = _lib.plcg_batch_add
plcg_batch_step = _lib.plcg_batch_step
plcg_batch_poll = _lib.plcg_batch_poll
plcg_batch_active = _lib.plcg_batch_active
plcg_batch_grid = _lib.plcg_batch_grid
plcg_batch_chunks_per_block = _lib.plcg_batch_chunks_per_block
plcg_batch_get_schedule = _lib.plcg_batch_get_schedule
plcg_batch_set_schedule = _lib.plcg_batch_set_schedule
plcg_batch_autotune = _lib.plcg_batch_autotune
plcg_batch_destroy = _lib.plcg_batch_destroy
plcg_batch_register = _lib.plcg_batch_register
plcg_batch_request_footprint = _lib.plcg_batch_request_footprint
plcg_batch_add_op = _lib.plcg_batch_add_op
plcg_serve = _lib.plcg_serve


class PlcgError(RuntimeError):
    def __init__(self, status, where):
        msg = plcg_last_error()
        super().__init__(f"{where} failed with status {status}: "
                         f"{msg.decode() if msg else ''}")
        self.status = status


def check(status, where):
    if status < 0:
        raise PlcgError(status, where)
    return status


def _dims_desc(kind, dims, diag=None, csr=None, jacobi=False, coef=None):
    dims = tuple(int(d) for d in dims)
    cx, cy, cz = coef if coef is not None else (None, None, None)
    if kind in ("2d5", PLCG_OP_STENCIL2D5):
        return plcg_operator_desc(PLCG_OP_STENCIL2D5, dims[0], dims[1], 1, None, 0, None, None,
                                  None, 1 if jacobi else 0, cx, cy, cz)
    if kind in ("3d7", PLCG_OP_STENCIL3D7):
        return plcg_operator_desc(PLCG_OP_STENCIL3D7, dims[0], dims[1], dims[2], None, 0, None,
                                  None, None, 1 if jacobi else 0, cx, cy, cz)
    dims = dims + (1,) * (3 - len(dims))
    if kind in ("diag", PLCG_OP_DIAG):
        return plcg_operator_desc(PLCG_OP_DIAG, dims[0], dims[1], dims[2], diag)
    if kind in ("csr", PLCG_OP_CSR):
        rowptr, colind, vals, nnz = csr if csr is not None else (None, None, None, 0)
        return plcg_operator_desc(PLCG_OP_CSR, dims[0], dims[1], dims[2], None, int(nnz),
                                  rowptr, colind, vals, 1 if jacobi else 0)
    raise ValueError(f"unknown operator kind {kind!r}")


def resident_supported(kind, n, method="plcg", l=1):
    """plcg_resident_supported for a kind name ("2d5", "3d7", "diag", "csr") or code."""
    code = {"2d5": PLCG_OP_STENCIL2D5, "3d7": PLCG_OP_STENCIL3D7, "diag": PLCG_OP_DIAG,
            "csr": PLCG_OP_CSR}.get(kind, kind)
    m = PLCG_METHOD_CG if method == "cg" else PLCG_METHOD_PLCG
    return plcg_resident_supported(int(code), int(n), m, int(l)) == 1


def _vec(v, n, name):
    """A device address from an int, or from a contiguous float64 GPU tensor of n
    elements (anything with data_ptr(), dtype, is_cuda, numel, is_contiguous)."""
    if v is None or isinstance(v, int):
        return v
    if not hasattr(v, "data_ptr"):
        raise TypeError(f"{name}: expected a device address or a tensor")
    if str(v.dtype) != "torch.float64" or not v.is_cuda or not v.is_contiguous():
        raise ValueError(f"{name}: needs a contiguous float64 tensor on the GPU")
    if n is not None and v.numel() != n:
        raise ValueError(f"{name}: has {v.numel()} elements, the operator has {n}")
    return v.data_ptr()


def _stream(stream):
    """None: torch's current stream on the current device (0 if torch is absent)."""
    if stream is not None:
        return stream
    try:
        import torch
        return torch.cuda.current_stream().cuda_stream
    except Exception:
        return 0


class Solver:
    """Convenience owner of one plcg_handle.  b and x may be given as device
    addresses or as contiguous float64 GPU tensors; stream None means torch's
    current stream."""

    def __init__(self, kind, dims, method="plcg", l=1, lmin=0.0, lmax=8.0, shifts=None,
                 check_every=0, max_restarts=-1, history_cap=0, precision="fp64",
                 inner_tol=0.0, diag=None, csr=None, jacobi=False, launch="auto",
                 x_update="auto", coef=None):
        """kind "2d5", "3d7", "diag" or "csr"; for "diag", `diag` is the device
        address of the n FP64 diagonal entries; for "csr", `csr` is (rowptr,
        colind, vals, nnz) with device addresses of int64 / int32 / FP64 arrays
        (copied by plcg_create); for "2d5" / "3d7", `coef` = (cx, cy, cz) device
        addresses of edge coefficients (cz None in 2D) makes the operator the
        variable-coefficient one; jacobi=True solves a CSR matrix or a
        variable-coefficient stencil Jacobi-preconditioned.
        launch: "auto", "streaming" or "resident" (PLCG_LAUNCH_*); x_update: "auto",
        "every" or "paired" (PLCG_X_*)."""
        self.desc = _dims_desc(kind, dims, diag, csr, jacobi, coef)
        self._shifts = None
        sp = None
        if shifts is not None:
            self._shifts = (ctypes.c_double * len(shifts))(*shifts)
            sp = ctypes.cast(self._shifts, ctypes.POINTER(ctypes.c_double))
        m = PLCG_METHOD_CG if method == "cg" else PLCG_METHOD_PLCG
        prec = PLCG_PREC_FP32_REFINED if precision == "fp32" else PLCG_PREC_FP64
        self.cfg = plcg_config(m, int(l), float(lmin), float(lmax), sp, int(check_every),
                               int(max_restarts), int(history_cap), prec, float(inner_tol),
                               LAUNCH_MODES[launch], X_UPDATES[x_update])
        self.method = method
        self.l = int(l)
        self.handle = _h()
        check(plcg_create(ctypes.byref(self.desc), ctypes.byref(self.cfg),
                          ctypes.byref(self.handle)), "plcg_create")
        self.n = plcg_size(self.handle)

    def solve(self, b, x, tol, maxit, stream=None):
        res = plcg_result()
        st = plcg_solve(self.handle, _vec(b, self.n, "b"), _vec(x, self.n, "x"), float(tol),
                        int(maxit), _stream(stream), ctypes.byref(res))
        check(st, "plcg_solve")
        return res

    def submit(self, b, x, tol, maxit, stream=None):
        """b and x must stay alive until poll() returns a result."""
        t = ctypes.c_uint64(0)
        check(plcg_submit(self.handle, _vec(b, self.n, "b"), _vec(x, self.n, "x"), float(tol),
                          int(maxit), _stream(stream), ctypes.byref(t)), "plcg_submit")
        return t.value

    def poll(self, ticket):
        res = plcg_result()
        st = plcg_poll(self.handle, ticket, ctypes.byref(res))
        if st == PLCG_NOT_READY:
            return None
        check(st, "plcg_poll")
        return res

    def apply(self, x, y, stream=None):
        check(plcg_apply(self.handle, _vec(x, self.n, "x"), _vec(y, self.n, "y"),
                         _stream(stream)), "plcg_apply")

    def shifts(self):
        out = (ctypes.c_double * max(self.l, 1))()
        check(plcg_get_shifts(self.handle, out), "plcg_get_shifts")
        return list(out)[: self.l]

    def history(self, cap):
        out = (ctypes.c_double * (4 * cap))()
        cnt = ctypes.c_int32(0)
        check(plcg_get_history(self.handle, out, cap, ctypes.byref(cnt)), "plcg_get_history")
        return [tuple(out[4 * k: 4 * k + 4]) for k in range(cnt.value)]

    def set_timing(self, on):
        check(plcg_set_timing(self.handle, 1 if on else 0), "plcg_set_timing")

    def close(self):
        if self.handle:
            plcg_destroy(self.handle)
            self.handle = _h()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _dptr(a):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def system_desc(dims, cx=None, cy=None, cz=None):
    """plcg_system_desc for host numpy coefficient arrays (kept alive by the caller)."""
    dims = tuple(int(d) for d in dims)
    kind = PLCG_OP_STENCIL2D5 if len(dims) == 2 else PLCG_OP_STENCIL3D7
    nz = dims[2] if len(dims) == 3 else 1
    return plcg_system_desc(kind, dims[0], dims[1], nz, _dptr(cx), _dptr(cy), _dptr(cz))


class Batch:
    """Convenience owner of one plcg_batch."""

    def __init__(self, l=2, max_slots=64, arena_bytes=1 << 30, chunks_per_block=0,
                 lmin=0.0, lmax=0.0, max_restarts=-1, use_graph=False, precision="fp64",
                 inner_tol=0.0):
        """precision "fp64", or "fp32" for FP32-stored inner solves inside FP64
        iterative refinement (inner_tol: the inner solves' relative tolerance)."""
        prec = PLCG_PREC_FP32_REFINED if precision == "fp32" else PLCG_PREC_FP64
        cfg = plcg_batch_config(int(l), float(lmin), float(lmax), int(max_slots),
                                int(arena_bytes), int(chunks_per_block), int(max_restarts),
                                1 if use_graph else 0, prec, float(inner_tol))
        self.handle = _h()
        check(plcg_batch_create(ctypes.byref(cfg), ctypes.byref(self.handle)), "plcg_batch_create")
        self._keep = {}

    def footprint(self, dims, cx=None, cy=None, cz=None):
        d = system_desc(dims, cx, cy, cz)
        return plcg_batch_footprint(self.handle, ctypes.byref(d))

    def add(self, dims, b_ptr, x_ptr, tol, maxit, stream=0, cx=None, cy=None, cz=None):
        """Ticket, or None when the batch has no room (PLCG_E_BUSY)."""
        d = system_desc(dims, cx, cy, cz)
        t = ctypes.c_uint64(0)
        st = plcg_batch_add(self.handle, ctypes.byref(d), b_ptr, x_ptr, float(tol), int(maxit),
                            stream, ctypes.byref(t))
        if st == PLCG_E_BUSY:
            return None
        check(st, "plcg_batch_add")
        return t.value

    def register(self, dims, cx=None, cy=None, cz=None, stream=0):
        d = system_desc(dims, cx, cy, cz)
        op = ctypes.c_int32(-1)
        check(plcg_batch_register(self.handle, ctypes.byref(d), stream, ctypes.byref(op)),
              "plcg_batch_register")
        return op.value

    def request_footprint(self, op_id, internal_x=True):
        return plcg_batch_request_footprint(self.handle, int(op_id), 1 if internal_x else 0)

    def add_op(self, op_id, b_ptr, x_ptr, tol, maxit, stream=0):
        t = ctypes.c_uint64(0)
        st = plcg_batch_add_op(self.handle, int(op_id), b_ptr, x_ptr, float(tol), int(maxit),
                               stream, ctypes.byref(t))
        if st == PLCG_E_BUSY:
            return None
        check(st, "plcg_batch_add_op")
        return t.value

    def serve(self, op_ids, b_ptrs, requests, ticks_per_round=16, time_limit_s=60.0, stream=0):
        """requests: list of (arrival_s, system, maxit, tol) or (arrival_s, system,
        maxit, tol, x_ptr) with x_ptr the device address receiving the solution
        (None: kept inside the batch), sorted by arrival.  Returns the list of
        plcg_request_outcome."""
        n = len(op_ids)
        ops = (ctypes.c_int32 * n)(*op_ids)
        bp = (ctypes.c_void_p * n)(*b_ptrs)
        rq = (plcg_request * len(requests))(*[plcg_request(float(r[0]), int(r[1]), int(r[2]),
                                                           float(r[3]),
                                                           r[4] if len(r) > 4 else None)
                                              for r in requests])
        out = (plcg_request_outcome * len(requests))()
        check(plcg_serve(self.handle, ops, bp, n, rq, len(requests), int(ticks_per_round),
                         float(time_limit_s), stream, out), "plcg_serve")
        return list(out)

    def step(self, ticks, stream=0):
        check(plcg_batch_step(self.handle, int(ticks), stream), "plcg_batch_step")

    def poll(self, ticket):
        res = plcg_result()
        st = plcg_batch_poll(self.handle, ticket, ctypes.byref(res))
        if st == PLCG_NOT_READY:
            return None
        check(st, "plcg_batch_poll")
        return res

    def active(self):
        return plcg_batch_active(self.handle)

    def grid(self):
        return plcg_batch_grid(self.handle)

    def chunks_per_block(self):
        return plcg_batch_chunks_per_block(self.handle)

    def schedule(self):
        """Chunks per streaming workgroup for systems of <= 8, <= 64 and more chunks."""
        out = (ctypes.c_int32 * 3)()
        check(plcg_batch_get_schedule(self.handle, out), "plcg_batch_get_schedule")
        return list(out)

    def set_schedule(self, cpb):
        """Chunks per workgroup by size class for systems admitted from now on."""
        check(plcg_batch_set_schedule(self.handle, (ctypes.c_int32 * 3)(*cpb)),
              "plcg_batch_set_schedule")

    def autotune(self, ticks, stream=0):
        check(plcg_batch_autotune(self.handle, int(ticks), stream), "plcg_batch_autotune")

    def close(self):
        if self.handle:
            plcg_batch_destroy(self.handle)
            self.handle = _h()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
