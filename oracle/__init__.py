"""ctypes front end of the FP64 CPU oracle (``hprlp_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the benchmark's
CPU-baseline leg, never by the library or its Python binding.  Nothing here touches the GPU
library, and the GPU library shares no code with it.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "hprlp_oracle.c")
LIB = os.path.join(HERE, "libhprlp_oracle.so")
LIB_OMP = os.path.join(HERE, "libhprlp_oracle_omp.so")  # same source, -fopenmp (timing only)

# check-trace columns (one row per check), same order as the C enum
TRACE_COLS = ["k", "t", "r", "sigma", "merit", "merit0", "merit_prev", "rel_p", "rel_d",
              "rel_gap", "pobj", "dobj", "dx", "dy", "err_p", "err_d", "restart",
              "sigma_new"]

STATUS = {1: "OPTIMAL", 2: "ITER_LIMIT", 3: "TIME_LIMIT", 4: "NUMERICAL"}


class Opts(C.Structure):
    _fields_ = [("tol", C.c_double), ("check_every", C.c_longlong),
                ("max_iter", C.c_longlong), ("time_limit", C.c_double),
                ("alpha1", C.c_double), ("alpha2", C.c_double), ("alpha3", C.c_double),
                ("sigma0", C.c_double), ("ruiz_iters", C.c_int),
                ("pock_chambolle", C.c_int), ("normalize_bc", C.c_int),
                ("power_max_iter", C.c_int), ("power_tol", C.c_double),
                ("lambda_override", C.c_double), ("use_halpern", C.c_int),
                ("rho", C.c_double), ("use_restart", C.c_int), ("sigma_update", C.c_int),
                ("trace_every_iter", C.c_int), ("t1_zero", C.c_int)]


class Result(C.Structure):
    _fields_ = [("iters", C.c_longlong), ("restarts", C.c_longlong), ("status", C.c_int),
                ("power_iters", C.c_int), ("sigma", C.c_double), ("lambda_", C.c_double),
                ("rel_p", C.c_double), ("rel_d", C.c_double), ("rel_gap", C.c_double),
                ("pobj", C.c_double), ("dobj", C.c_double), ("beta_b", C.c_double),
                ("beta_c", C.c_double), ("t_power", C.c_double), ("t_solve", C.c_double),
                ("n_checks", C.c_longlong), ("n_iter_trace", C.c_longlong)]


DEFAULTS = dict(tol=1e-8, check_every=150, max_iter=1_000_000, time_limit=0.0, alpha1=0.2,
                alpha2=0.6, alpha3=0.2, sigma0=1.0, ruiz_iters=10, pock_chambolle=1,
                normalize_bc=1, power_max_iter=5000, power_tol=1e-10, lambda_override=0.0,
                use_halpern=1, rho=2.0, use_restart=1, sigma_update=1, trace_every_iter=0,
                t1_zero=0)


_FLAGS = ["-O2", "-std=c11", "-D_POSIX_C_SOURCE=199309L", "-ffp-contract=off",
          "-fno-fast-math", "-fPIC", "-shared"]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain -O2, no fast-math, no FP contraction), and the same
    source with -fopenmp (bit-identical results on several threads; for timing)."""
    for lib, extra in ((LIB, []), (LIB_OMP, ["-fopenmp"])):
        if force or not os.path.exists(lib) or os.path.getmtime(lib) < os.path.getmtime(SRC):
            tmp = lib + ".tmp"
            subprocess.check_call(["gcc", *_FLAGS, *extra, SRC, "-o", tmp, "-lm"])
            os.replace(tmp, lib)
    return LIB


_libs = {}


def _load(threads: int = 1):
    """The plain build (threads = 1) or the OpenMP build set to `threads` threads."""
    key = "plain" if threads == 1 else "omp"
    if key not in _libs:
        build()
        lib = C.CDLL(LIB if key == "plain" else LIB_OMP)
        P = C.c_void_p
        lib.oracle_scale.argtypes = [C.c_longlong, C.c_longlong, P, P, P, P, P, P, P,
                                     C.POINTER(Opts), P, P, P, P, P, P, P,
                                     C.POINTER(C.c_double), C.POINTER(C.c_double)]
        lib.oracle_scale.restype = C.c_int
        lib.oracle_power.argtypes = [C.c_longlong, C.c_longlong, P, P, P, C.c_int, C.c_double,
                                     C.POINTER(C.c_double)]
        lib.oracle_power.restype = C.c_int
        lib.oracle_solve.argtypes = [C.c_longlong, C.c_longlong, C.c_longlong, P, P, P, P, P,
                                     P, P, C.POINTER(Opts), P, P, P, P, P, C.POINTER(Result),
                                     P, C.c_longlong, P, C.c_longlong, P]
        lib.oracle_solve.restype = C.c_int
        lib.oracle_set_threads.argtypes = [C.c_int]
        lib.oracle_set_threads.restype = C.c_int
        _libs[key] = lib
    lib = _libs[key]
    if key == "omp":
        lib.oracle_set_threads(int(threads))
    return lib


def _p(a: Optional[np.ndarray]):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


def _opts(**kw) -> Opts:
    d = dict(DEFAULTS)
    for k, v in kw.items():
        if k not in d:
            raise KeyError(f"unknown oracle option {k}")
        d[k] = v
    return Opts(**d)


def _csr(lp):
    return (np.ascontiguousarray(lp.rowptr, dtype=np.int64),
            np.ascontiguousarray(lp.colidx, dtype=np.int32),
            np.ascontiguousarray(lp.val, dtype=np.float64))


@dataclass
class Scaling:
    val: np.ndarray
    dr: np.ndarray
    dc: np.ndarray
    b: np.ndarray
    c: np.ndarray
    l: np.ndarray
    u: np.ndarray
    beta_b: float
    beta_c: float


def scale(lp, **kw) -> Scaling:
    """Preconditioning of Section 4.1 (Ruiz x10, Pock-Chambolle alpha=1, b/c normalisation)."""
    lib = _load()
    rp, ci, val = _csr(lp)
    m, n = lp.m, lp.n
    out = Scaling(np.empty(len(val)), np.empty(m), np.empty(n), np.empty(m), np.empty(n),
                  np.empty(n), np.empty(n), 0.0, 0.0)
    bb, bc = C.c_double(), C.c_double()
    o = _opts(**kw)
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (lp.b, lp.c, lp.l, lp.u)]
    rc = lib.oracle_scale(m, n, _p(rp), _p(ci), _p(val), *[_p(a) for a in arrs],
                          C.byref(o), _p(out.val), _p(out.dr), _p(out.dc), _p(out.b),
                          _p(out.c), _p(out.l), _p(out.u), C.byref(bb), C.byref(bc))
    if rc != 0:
        raise RuntimeError(f"oracle_scale failed ({rc})")
    out.beta_b, out.beta_c = bb.value, bc.value
    return out


def power(m, n, rowptr, colidx, val, max_iter=5000, tol=1e-10):
    """Power method for lambda_1(A A^T); returns (lambda, iterations)."""
    lib = _load()
    lam = C.c_double()
    rp = np.ascontiguousarray(rowptr, dtype=np.int64)
    ci = np.ascontiguousarray(colidx, dtype=np.int32)
    v = np.ascontiguousarray(val, dtype=np.float64)
    it = lib.oracle_power(m, n, _p(rp), _p(ci), _p(v), int(max_iter), float(tol),
                          C.byref(lam))
    return lam.value, it


@dataclass
class SolveResult:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    x_cur: np.ndarray
    y_cur: np.ndarray
    status: str
    iters: int
    restarts: int
    sigma: float
    lam: float
    power_iters: int
    rel_p: float
    rel_d: float
    rel_gap: float
    pobj: float
    dobj: float
    beta_b: float
    beta_c: float
    t_power: float
    t_solve: float
    trace: np.ndarray = field(repr=False)
    iter_trace: np.ndarray = field(repr=False)
    dr: np.ndarray = field(repr=False)
    dc: np.ndarray = field(repr=False)

    @property
    def rel_kkt(self) -> float:
        return max(self.rel_p, self.rel_d, self.rel_gap)

    def trace_col(self, name: str) -> np.ndarray:
        return self.trace[:, TRACE_COLS.index(name)]


def solve(lp, check_cap: int = 100000, iter_cap: int = 0, threads: int = 1,
          **kw) -> SolveResult:
    """Run HPR-LP (Algorithm 2) on the CPU.  Keyword options as in ``DEFAULTS``.
    threads > 1 runs the OpenMP build (same results bit for bit; for timing)."""
    lib = _load(threads)
    rp, ci, val = _csr(lp)
    m, n = lp.m, lp.n
    o = _opts(**kw)
    x, z, xc = np.empty(n), np.empty(n), np.empty(n)
    y, yc = np.empty(m), np.empty(m)
    trace = np.zeros((max(check_cap, 1), len(TRACE_COLS)))
    itr = np.zeros((max(iter_cap, 1), 4))
    sc = np.empty(m + n)
    res = Result()
    arrs = [np.ascontiguousarray(a, dtype=np.float64) for a in (lp.b, lp.c, lp.l, lp.u)]
    rc = lib.oracle_solve(lp.m1, lp.m2, n, _p(rp), _p(ci), _p(val), *[_p(a) for a in arrs],
                          C.byref(o), _p(x), _p(y), _p(z), _p(xc), _p(yc), C.byref(res),
                          _p(trace), check_cap, _p(itr), iter_cap, _p(sc))
    if rc != 0:
        raise RuntimeError(f"oracle_solve failed ({rc})")
    return SolveResult(x, y, z, xc, yc, STATUS.get(res.status, str(res.status)), res.iters,
                       res.restarts, res.sigma, res.lambda_, res.power_iters, res.rel_p,
                       res.rel_d, res.rel_gap, res.pobj, res.dobj, res.beta_b, res.beta_c,
                       res.t_power, res.t_solve, trace[:min(res.n_checks, check_cap)],
                       itr[:min(res.n_iter_trace, iter_cap)], sc[:m], sc[m:])
