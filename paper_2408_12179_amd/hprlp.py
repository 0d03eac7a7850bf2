"""Python binding of the HPR-LP C ABI (``include/hprlp.h``).

Argument marshalling only: every step of the solve runs in ``libhprlp.so`` (HIP kernels for
gfx950).  PyTorch provides the device workspace and the stream.  There is no CPU fallback:
if the library is not built, importing works but creating a solver raises.
"""
from __future__ import annotations

import ctypes as C
import os
from dataclasses import dataclass
from typing import Optional

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libhprlp.so")

OK, EINVAL, EDIM, ENONFINITE, EBOUNDS, ENOTLOSSLESS, ENOMEM, EHIP, ESTATE = \
    0, -1, -2, -3, -4, -5, -6, -7, -8
STATUS = {0: "UNSOLVED", 1: "OPTIMAL", 2: "ITER_LIMIT", 3: "TIME_LIMIT", 4: "NUMERICAL"}
FP64, MIXED, FP64_A32 = 0, 1, 2
XBAR, YBAR, ZBAR, XCUR, YCUR, DROW, DCOL = range(7)
TRACE_COLS = ["k", "t", "r", "sigma", "merit", "merit0", "merit_prev", "rel_p", "rel_d",
              "rel_gap", "pobj", "dobj", "dx", "dy", "err_p", "err_d", "restart",
              "sigma_new"]
BATCH_TRACE_COLS = ["k", "t", "r", "sigma", "merit", "rel_p", "rel_d", "rel_gap", "restart",
                    "sigma_new"]
EXPORTS = ["hprlp_default_options", "hprlp_workspace_bytes", "hprlp_workspace_bytes_batched",
           "hprlp_create", "hprlp_create_noalloc", "hprlp_create_batched", "hprlp_solve",
           "hprlp_stats",
           "hprlp_stats_instance", "hprlp_get_iterate", "hprlp_get_trace",
           "hprlp_get_trace_instance", "hprlp_get_schedule", "hprlp_begin", "hprlp_step",
           "hprlp_time_passes", "hprlp_plan_schedule", "hprlp_last_error", "hprlp_destroy"]


class Options(C.Structure):
    _fields_ = [("tol", C.c_double), ("check_every", C.c_longlong),
                ("max_iter", C.c_longlong), ("time_limit", C.c_double),
                ("alpha1", C.c_double), ("alpha2", C.c_double), ("alpha3", C.c_double),
                ("sigma0", C.c_double), ("ruiz_iters", C.c_int), ("pock_chambolle", C.c_int),
                ("normalize_bc", C.c_int), ("power_max_iter", C.c_int),
                ("power_tol", C.c_double), ("lambda_override", C.c_double),
                ("use_halpern", C.c_int), ("use_restart", C.c_int), ("sigma_update", C.c_int),
                ("precision", C.c_int), ("tol_switch", C.c_double),
                ("stall_checks", C.c_int), ("tile_nnz", C.c_int),
                ("tile_rows", C.c_int), ("short_max", C.c_int), ("split_len", C.c_int),
                ("chunk_nnz", C.c_int), ("reorder", C.c_int), ("profile", C.c_int),
                ("verbose", C.c_int), ("autotune", C.c_int), ("stall_ratio", C.c_double),
                ("graph", C.c_int), ("rho", C.c_double), ("t1_zero", C.c_int),
                ("setup_on_host", C.c_int), ("tile_order", C.c_int),
                ("bundle_rows", C.c_int)]


class Stats(C.Structure):
    _fields_ = [("iters", C.c_longlong), ("restarts", C.c_longlong),
                ("iters_fp32", C.c_longlong), ("status", C.c_int), ("power_iters", C.c_int),
                ("sigma", C.c_double), ("lambda_", C.c_double), ("rel_p", C.c_double),
                ("rel_d", C.c_double), ("rel_gap", C.c_double), ("pobj", C.c_double),
                ("dobj", C.c_double), ("beta_b", C.c_double), ("beta_c", C.c_double),
                ("t_power_ms", C.c_double), ("t_solve_ms", C.c_double),
                ("bytes_per_iter", C.c_double), ("col_pass_ms", C.c_double),
                ("row_pass_ms", C.c_double), ("col_pass_launches", C.c_longlong),
                ("row_pass_launches", C.c_longlong), ("split_ms", C.c_double),
                ("n_checks", C.c_longlong), ("n_compactions", C.c_longlong),
                ("t_setup_ms", C.c_double), ("t_prep_ms", C.c_double),
                ("t_tune_ms", C.c_double)]

    def as_dict(self) -> dict:
        d = {f: getattr(self, f) for f, _ in self._fields_}
        d["lambda"] = d.pop("lambda_")
        d["status"] = STATUS.get(d["status"], str(d["status"]))
        return d


class HPRLPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"hprlp error {code}: {msg}")
        self.code = code


_lib = None


def load() -> C.CDLL:
    """Load libhprlp.so (built in-tree by ``__graft_entry__.build()``); raise if missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library {LIB_PATH} is not built; run __graft_entry__.build()")
    lib = C.CDLL(LIB_PATH)
    P = C.c_void_p
    lib.hprlp_default_options.argtypes = [C.POINTER(Options)]
    lib.hprlp_default_options.restype = None
    lib.hprlp_workspace_bytes.argtypes = [C.c_int64, C.c_int64, C.c_int64, C.c_int64,
                                          C.POINTER(Options), C.POINTER(C.c_size_t)]
    lib.hprlp_create.argtypes = [C.POINTER(P), C.c_int64, C.c_int64, C.c_int64, P, P, P, P, P,
                                 P, P, C.POINTER(Options), P, C.c_size_t, P]
    lib.hprlp_create_noalloc.argtypes = [C.POINTER(P), C.c_int64, C.c_int64, C.c_int64, P, P,
                                         P, P, P, P, P, C.POINTER(Options), P]
    lib.hprlp_workspace_bytes_batched.argtypes = [C.c_int32, C.c_int64, C.c_int64, C.c_int64,
                                                  C.POINTER(Options), C.POINTER(C.c_size_t)]
    lib.hprlp_create_batched.argtypes = [C.POINTER(P), C.c_int32, P, P, P, P, P, P, P, P, P, P,
                                         P, C.POINTER(Options), P, C.c_size_t, P]
    lib.hprlp_stats_instance.argtypes = [P, C.c_int32, C.POINTER(Stats)]
    lib.hprlp_get_trace_instance.argtypes = [P, C.c_int32, P, C.c_longlong,
                                             C.POINTER(C.c_longlong)]
    lib.hprlp_get_schedule.argtypes = [P, C.c_int, P, P, C.POINTER(C.c_double)]
    lib.hprlp_plan_schedule.argtypes = [C.c_int64, C.c_int64, P, P, P, C.c_int, P]
    lib.hprlp_solve.argtypes = [P, P, P, P, C.POINTER(C.c_int)]
    lib.hprlp_begin.argtypes = [P]
    lib.hprlp_step.argtypes = [P, C.c_int]
    lib.hprlp_stats.argtypes = [P, C.POINTER(Stats)]
    lib.hprlp_get_iterate.argtypes = [P, C.c_int, P]
    lib.hprlp_get_trace.argtypes = [P, P, C.c_longlong, C.POINTER(C.c_longlong)]
    lib.hprlp_time_passes.argtypes = [P, C.c_int, C.POINTER(C.c_double), C.POINTER(C.c_double)]
    lib.hprlp_last_error.argtypes = [P]
    lib.hprlp_last_error.restype = C.c_char_p
    lib.hprlp_destroy.argtypes = [P]
    lib.hprlp_destroy.restype = None
    for name in EXPORTS:
        if name not in ("hprlp_default_options", "hprlp_last_error", "hprlp_destroy"):
            getattr(lib, name).restype = C.c_int
    _lib = lib
    return lib


def default_options(**kw) -> Options:
    o = Options()
    load().hprlp_default_options(C.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise KeyError(f"unknown option {k}")
        setattr(o, k, v)
    return o


def _ptr(a: Optional[np.ndarray]):
    return None if a is None else C.c_void_p(a.ctypes.data)


def last_error(handle=None) -> str:
    return load().hprlp_last_error(handle).decode()


def workspace_bytes(m1: int, m2: int, n: int, nnz: int, opts: Options) -> int:
    out = C.c_size_t()
    rc = load().hprlp_workspace_bytes(m1, m2, n, nnz, C.byref(opts), C.byref(out))
    if rc != OK:
        raise HPRLPError(rc, last_error())
    return int(out.value)


def plan_schedule(lp, matrix: int, **options) -> dict:
    """Schedule counts hprlp_create would build for A (matrix=0) or A^T (matrix=1) of lp,
    computed on the host (no GPU)."""
    opts = default_options(**options)
    rowptr = np.ascontiguousarray(lp.rowptr, dtype=np.int64)
    colidx = np.ascontiguousarray(lp.colidx, dtype=np.int32)
    counts = np.zeros(6, dtype=np.int64)
    rc = load().hprlp_plan_schedule(lp.m, lp.n, _ptr(rowptr), _ptr(colidx), C.byref(opts),
                                    matrix, _ptr(counts))
    if rc != OK:
        raise HPRLPError(rc, last_error())
    return dict(items=int(counts[0]), tiles=int(counts[1]), row_items=int(counts[2]),
                chunks=int(counts[3]), bundle_items=int(counts[5]))


def workspace_bytes_batched(n_inst: int, m: int, n: int, nnz: int, opts: Options) -> int:
    out = C.c_size_t()
    rc = load().hprlp_workspace_bytes_batched(n_inst, m, n, nnz, C.byref(opts), C.byref(out))
    if rc != OK:
        raise HPRLPError(rc, last_error())
    return int(out.value)


@dataclass
class Solution:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    status: str
    stats: dict


class Solver:
    """One LP on one GPU.  ``lp`` is any object with m1, m2, n, rowptr, colidx, val, b, c, l,
    u attributes (e.g. ``lpgen.LP``); options are the fields of ``hprlp_options``.

    ``batched=True`` solves the independent LPs packed block-diagonally in ``lp`` (which then
    also carries inst_row_off, inst_col_off, inst_m1) in one run; ``lambdas`` optionally
    gives lambda per instance."""

    def __init__(self, lp, device: int = 0, batched: bool = False, lambdas=None, **options):
        import torch  # device memory and stream only
        lib = load()
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the HPR-LP library runs on an MI355X only")
        self._lib = lib
        self._h = None
        self.batched = batched
        self.m1, self.m2, self.n = int(lp.m1), int(lp.m2), int(lp.n)
        self.m = self.m1 + self.m2
        self._arrays = [np.ascontiguousarray(lp.rowptr, dtype=np.int64),
                        np.ascontiguousarray(lp.colidx, dtype=np.int32)] + \
            [np.ascontiguousarray(a, dtype=np.float64) for a in (lp.val, lp.b, lp.c, lp.l, lp.u)]
        self.opts = default_options(**options)
        nnz = int(self._arrays[0][-1])
        if batched:
            self._inst = [np.ascontiguousarray(a, dtype=np.int64)
                          for a in (lp.inst_row_off, lp.inst_col_off, lp.inst_m1)]
            self.n_inst = len(self._inst[2])
            self._lams = None if lambdas is None else \
                np.ascontiguousarray(lambdas, dtype=np.float64)
            if self._lams is not None and len(self._lams) != self.n_inst:
                raise ValueError("lambdas needs one value per instance")
            nbytes = workspace_bytes_batched(self.n_inst, self.m, self.n, nnz, self.opts)
        else:
            self.n_inst = 1
            nbytes = workspace_bytes(self.m1, self.m2, self.n, nnz, self.opts)
        self.device = torch.device("cuda", device)
        self._ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        self._stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        ws = C.c_void_p(self._ws.data_ptr())
        stream = C.c_void_p(self._stream.cuda_stream)
        if batched:
            rc = lib.hprlp_create_batched(C.byref(h), self.n_inst, *[_ptr(a) for a in self._inst],
                                          *[_ptr(a) for a in self._arrays], _ptr(self._lams),
                                          C.byref(self.opts), ws, nbytes, stream)
        else:
            rc = lib.hprlp_create(C.byref(h), self.m1, self.m2, self.n,
                                  *[_ptr(a) for a in self._arrays], C.byref(self.opts), ws,
                                  nbytes, stream)
        if rc != OK:
            raise HPRLPError(rc, last_error())
        self._h = h
        self.workspace_bytes = nbytes

    def _check(self, rc):
        if rc != OK:
            raise HPRLPError(rc, self._lib.hprlp_last_error(self._h).decode())

    def solve(self) -> Solution:
        x, z = np.empty(self.n), np.empty(self.n)
        y = np.empty(self.m)
        st = C.c_int()
        self._check(self._lib.hprlp_solve(self._h, _ptr(x), _ptr(y), _ptr(z), C.byref(st)))
        return Solution(x, y, z, STATUS.get(st.value, str(st.value)), self.stats())

    def solve_device(self):
        """Solve and return (x, y, z) as torch tensors on the GPU (outputs written on device)."""
        import torch
        x = torch.empty(self.n, dtype=torch.float64, device=self.device)
        z = torch.empty(self.n, dtype=torch.float64, device=self.device)
        y = torch.empty(self.m, dtype=torch.float64, device=self.device)
        st = C.c_int()
        self._check(self._lib.hprlp_solve(self._h, C.c_void_p(x.data_ptr()),
                                          C.c_void_p(y.data_ptr()), C.c_void_p(z.data_ptr()),
                                          C.byref(st)))
        return x, y, z, STATUS.get(st.value, str(st.value))

    def stats(self) -> dict:
        s = Stats()
        self._check(self._lib.hprlp_stats(self._h, C.byref(s)))
        return s.as_dict()

    def stats_instance(self, i: int) -> dict:
        s = Stats()
        self._check(self._lib.hprlp_stats_instance(self._h, i, C.byref(s)))
        return s.as_dict()

    def trace_instance(self, i: int) -> np.ndarray:
        n = C.c_longlong()
        self._check(self._lib.hprlp_get_trace_instance(self._h, i, None, 0, C.byref(n)))
        out = np.zeros((n.value, len(BATCH_TRACE_COLS)))
        self._check(self._lib.hprlp_get_trace_instance(self._h, i, _ptr(out), n.value,
                                                       C.byref(n)))
        return out

    def iterate(self, which: int) -> np.ndarray:
        size = self.m if which in (YBAR, YCUR, DROW) else self.n
        out = np.empty(size)
        self._check(self._lib.hprlp_get_iterate(self._h, which, _ptr(out)))
        return out

    def trace(self) -> np.ndarray:
        n = C.c_longlong()
        self._check(self._lib.hprlp_get_trace(self._h, None, 0, C.byref(n)))
        out = np.zeros((n.value, len(TRACE_COLS)))
        self._check(self._lib.hprlp_get_trace(self._h, _ptr(out), n.value, C.byref(n)))
        return out

    def schedule(self, matrix: int) -> dict:
        """Schedule of A (matrix=0, row pass) or A^T (matrix=1, column pass)."""
        params = np.zeros(5, dtype=np.int32)
        counts = np.zeros(6, dtype=np.int64)
        ms = C.c_double()
        self._check(self._lib.hprlp_get_schedule(self._h, matrix, _ptr(params), _ptr(counts),
                                                 C.byref(ms)))
        keys = ("tile_nnz", "tile_rows", "short_max", "split_len", "chunk_nnz")
        d = {k: int(v) for k, v in zip(keys, params)}
        d.update(items=int(counts[0]), tiles=int(counts[1]), row_items=int(counts[2]),
                 chunks=int(counts[3]), column_order=bool(counts[4]),
                 bundle_items=int(counts[5]), tuned_ms=ms.value)
        return d

    def begin(self) -> dict:
        """Start a solve without iterating (lambda, sigma0, the origin); returns the stats."""
        self._check(self._lib.hprlp_begin(self._h))
        return self.stats()

    def step(self, iters: int):
        """Advance from the current state (after begin or a solve): a single LP runs `iters`
        plain iterations (no checks); a batch runs iters / check_every whole chunks with
        their checks and decisions."""
        self._check(self._lib.hprlp_step(self._h, iters))

    def time_passes(self, reps: int = 50):
        a, b = C.c_double(), C.c_double()
        self._check(self._lib.hprlp_time_passes(self._h, reps, C.byref(a), C.byref(b)))
        return a.value, b.value

    def close(self):
        if getattr(self, "_h", None):
            self._lib.hprlp_destroy(self._h)
            self._h = None
            self._ws = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
