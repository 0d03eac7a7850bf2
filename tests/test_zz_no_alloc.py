"""hprlp_create_noalloc (the create that allocates nothing: its workspace is the library's
static per-device scratch) against hprlp_create with a caller workspace, through the C ABI.

Two create/solve/destroy rounds in a row on one device, the second on a smaller LP, so the
second runs in scratch that still holds the first problem's data.  The bar is the one every
GPU path meets against the path it varies: the same kernels on the same inputs, so the
returned x, y, z, the check trace and the iteration counts must be identical bit for bit.
Also: a second live handle on the same device is refused (ESTATE), a problem above the
scratch size is refused (EINVAL) before any GPU work, and profile / autotune are refused.
"""
import ctypes as C

import numpy as np
import pytest

import lpgen
from paper_2408_12179_amd import hprlp

pytestmark = pytest.mark.gpu


def _create_noalloc(lib, lp, opts):
    arrs = [np.ascontiguousarray(lp.rowptr, dtype=np.int64),
            np.ascontiguousarray(lp.colidx, dtype=np.int32)] + \
        [np.ascontiguousarray(a, dtype=np.float64) for a in (lp.val, lp.b, lp.c, lp.l, lp.u)]
    h = C.c_void_p()
    rc = lib.hprlp_create_noalloc(C.byref(h), lp.m1, lp.m2, lp.n,
                                  *[C.c_void_p(a.ctypes.data) for a in arrs], C.byref(opts),
                                  None)
    return rc, h, arrs


def _solve(lib, h, m, n):
    x, y, z = np.empty(n), np.empty(m), np.empty(n)
    st = C.c_int()
    rc = lib.hprlp_solve(h, C.c_void_p(x.ctypes.data), C.c_void_p(y.ctypes.data),
                         C.c_void_p(z.ctypes.data), C.byref(st))
    assert rc == 0, hprlp.last_error(h)
    s = hprlp.Stats()
    assert lib.hprlp_stats(h, C.byref(s)) == 0
    n_rows = C.c_longlong()
    assert lib.hprlp_get_trace(h, None, 0, C.byref(n_rows)) == 0
    tr = np.zeros((n_rows.value, len(hprlp.TRACE_COLS)))
    assert lib.hprlp_get_trace(h, C.c_void_p(tr.ctypes.data), n_rows.value,
                               C.byref(n_rows)) == 0
    return x, y, z, st.value, s.as_dict(), tr


def test_noalloc_matches_workspace_create_twice():
    import torch
    torch.cuda.init()
    lib = hprlp.load()
    big = lpgen.make("zipf1m", scale=0.01)           # ~112k nonzeros
    small = lpgen.make("tiny")                       # ~1k nonzeros, second call
    for lp in (big, small):
        ref = hprlp.Solver(lp, max_iter=3000)
        rs = ref.solve()
        rtr = ref.trace()
        ref.close()
        opts = hprlp.default_options(max_iter=3000)
        rc, h, keep = _create_noalloc(lib, lp, opts)
        assert rc == 0, hprlp.last_error()
        try:
            # the scratch is taken while this handle lives
            rc2, h2, _ = _create_noalloc(lib, lp, opts)
            assert rc2 == hprlp.ESTATE and not h2.value
            x, y, z, st, stats, tr = _solve(lib, h, lp.m, lp.n)
        finally:
            lib.hprlp_destroy(h)
        np.testing.assert_array_equal(x, rs.x)
        np.testing.assert_array_equal(y, rs.y)
        np.testing.assert_array_equal(z, rs.z)
        np.testing.assert_array_equal(tr, rtr)
        assert hprlp.STATUS[st] == rs.status
        assert stats["iters"] == rs.stats["iters"] and stats["restarts"] == rs.stats["restarts"]
        print(lp.name, rs.status, stats["iters"], "iterations: identical")


def test_noalloc_refusals():
    lib = hprlp.load()
    lp = lpgen.make("tiny")
    for kw in (dict(profile=10), dict(autotune=1)):
        rc, h, _ = _create_noalloc(lib, lp, hprlp.default_options(**kw))
        assert rc == hprlp.EINVAL and not h.value, kw
    # above the scratch: refused from the sizes alone
    big = lpgen.make("zipf1m", scale=0.5)
    rc, h, _ = _create_noalloc(lib, big, hprlp.default_options())
    assert rc == hprlp.EINVAL and not h.value
    assert "static scratch" in hprlp.last_error()
