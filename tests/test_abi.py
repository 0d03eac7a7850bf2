"""The C ABI without a GPU: exported symbols, struct layouts, defaults and input validation
(every validation error is returned before any HIP call, so these run on the CPU)."""
import ctypes as C
import os
import re
import subprocess

import numpy as np
import pytest

import lpgen
from paper_2408_12179_amd import hprlp

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hprlp.h")


@pytest.fixture(scope="module")
def lib():
    return hprlp.load()


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hprlp_[a-z_]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert "hprlp_create" in names and "hprlp_solve" in names and "hprlp_stats" in names
    for name in names:
        assert hasattr(lib, name), name
    assert sorted(hprlp.EXPORTS) == names


def test_struct_layout_matches_header(tmp_path):
    src = tmp_path / "layout.c"
    fields_o = [f for f, _ in hprlp.Options._fields_]
    fields_s = [f if f != "lambda_" else "lambda" for f, _ in hprlp.Stats._fields_]
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "hprlp.h"', 'int main(void){',
             'printf("%zu %zu\\n", sizeof(hprlp_options), sizeof(hprlp_stats_t));']
    lines += [f'printf("%zu\\n", offsetof(hprlp_options, {f}));' for f in fields_o]
    lines += [f'printf("%zu\\n", offsetof(hprlp_stats_t, {f}));' for f in fields_s]
    lines += ["return 0;}"]
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.check_call(["gcc", "-std=c99", "-I", os.path.dirname(HEADER), str(src), "-o", str(exe)])
    out = [int(v) for v in subprocess.check_output([str(exe)]).split()]
    assert out[0] == C.sizeof(hprlp.Options) and out[1] == C.sizeof(hprlp.Stats)
    offs = out[2:]
    want = [getattr(hprlp.Options, f).offset for f in fields_o] + \
           [getattr(hprlp.Stats, f if f != "lambda" else "lambda_").offset for f in fields_s]
    assert offs == want


def test_default_options_are_the_papers(lib):
    o = hprlp.default_options()
    assert o.tol == 1e-8 and o.check_every == 150
    assert (o.alpha1, o.alpha2, o.alpha3) == (0.2, 0.6, 0.2)
    assert o.sigma0 == 1.0 and o.ruiz_iters == 10 and o.pock_chambolle == 1
    assert o.normalize_bc == 1 and o.use_halpern == 1 and o.use_restart == 1
    assert o.sigma_update == 1 and o.precision == hprlp.FP64 and o.tol_switch == 1e-5
    assert o.tile_nnz > 0 and o.split_len >= o.short_max


def test_workspace_bytes(lib):
    o = hprlp.default_options()
    a = hprlp.workspace_bytes(50, 50, 200, 1000, o)
    b = hprlp.workspace_bytes(500, 500, 2000, 10000, o)
    assert 0 < a < b
    o2 = hprlp.default_options(precision=hprlp.MIXED)
    assert hprlp.workspace_bytes(500, 500, 2000, 10000, o2) > 0
    with pytest.raises(hprlp.HPRLPError) as e:
        hprlp.workspace_bytes(0, 0, 10, 10, o)
    assert e.value.code == hprlp.EDIM


def _create(lib, lp, ws=256, **opt):
    o = hprlp.default_options(**opt)
    arrs = [np.ascontiguousarray(lp.rowptr, dtype=np.int64),
            np.ascontiguousarray(lp.colidx, dtype=np.int32)] + \
        [np.ascontiguousarray(a, dtype=np.float64) for a in (lp.val, lp.b, lp.c, lp.l, lp.u)]
    h = C.c_void_p()
    rc = lib.hprlp_create(C.byref(h), lp.m1, lp.m2, lp.n, *[C.c_void_p(a.ctypes.data) for a in arrs],
                          C.byref(o), C.c_void_p(ws), 1 << 30, None)
    return rc, lib.hprlp_last_error(None).decode()


def _bad(mutate):
    lp = lpgen.make("tiny")
    lp = lpgen.LP(lp.name, lp.m1, lp.m2, lp.n, lp.rowptr.copy(), lp.colidx.copy(), lp.val.copy(),
                  lp.b.copy(), lp.c.copy(), lp.l.copy(), lp.u.copy())
    mutate(lp)
    return lp


@pytest.mark.parametrize("case,code", [
    ("empty_rows", hprlp.EDIM),
    ("rowptr_not_monotone", hprlp.EDIM),
    ("col_out_of_range", hprlp.EDIM),
    ("repeated_col", hprlp.EDIM),
    ("nan_in_A", hprlp.ENONFINITE),
    ("inf_in_b", hprlp.ENONFINITE),
    ("nan_bound", hprlp.ENONFINITE),
    ("l_gt_u", hprlp.EBOUNDS),
    ("l_plus_inf", hprlp.EBOUNDS),
    ("not_fp32_exact", hprlp.ENOTLOSSLESS),
    ("bad_option", hprlp.EINVAL),
    ("misaligned_workspace", hprlp.EINVAL),
    ("null_workspace", hprlp.EINVAL),
])
def test_create_rejects_bad_input_before_any_gpu_call(lib, case, code):
    opt, ws = {}, 256
    if case == "empty_rows":
        lp = _bad(lambda p: None)
        lp.m1, lp.m2 = 0, 0
        lp.rowptr = lp.rowptr[:1]
    elif case == "rowptr_not_monotone":
        lp = _bad(lambda p: p.rowptr.__setitem__(3, p.rowptr[4] + 1))
    elif case == "col_out_of_range":
        lp = _bad(lambda p: p.colidx.__setitem__(5, p.n))
    elif case == "repeated_col":
        lp = _bad(lambda p: p.colidx.__setitem__(p.rowptr[0] + 1, p.colidx[p.rowptr[0]]))
    elif case == "nan_in_A":
        lp = _bad(lambda p: p.val.__setitem__(7, np.nan))
    elif case == "inf_in_b":
        lp = _bad(lambda p: p.b.__setitem__(2, np.inf))
    elif case == "nan_bound":
        lp = _bad(lambda p: p.u.__setitem__(2, np.nan))
    elif case == "l_gt_u":
        lp = _bad(lambda p: (p.l.__setitem__(4, 5.0), p.u.__setitem__(4, 1.0)))
    elif case == "l_plus_inf":
        lp = _bad(lambda p: (p.l.__setitem__(4, np.inf), p.u.__setitem__(4, np.inf)))
    elif case == "not_fp32_exact":
        lp = _bad(lambda p: p.val.__setitem__(0, 0.1))
        opt = dict(precision=hprlp.MIXED)
    elif case == "bad_option":
        lp = _bad(lambda p: None)
        opt = dict(tol=0.0)
    elif case == "misaligned_workspace":
        lp = _bad(lambda p: None)
        ws = 257
    else:
        lp = _bad(lambda p: None)
        ws = 0
    rc, msg = _create(lib, lp, ws=ws, **opt)
    assert rc == code, (rc, msg)
    assert msg


def test_repeated_columns_in_unsorted_rows(lib):
    # rows whose columns strictly increase skip the marker check; an unsorted row goes
    # through it: a repeat there is refused, an unsorted row without one is accepted (the
    # misaligned workspace is then the first thing create refuses)
    def permute_row(p, repeat):
        a, e = p.rowptr[3], p.rowptr[4]
        assert e - a >= 3
        cols = p.colidx[a:e][::-1].copy()          # reversed: not increasing
        if repeat:
            cols[-1] = cols[0]                     # first and last entry, not adjacent
        p.colidx[a:e] = cols
    rc, msg = _create(lib, _bad(lambda p: permute_row(p, True)), ws=256)
    assert rc == hprlp.EDIM and "repeated column" in msg, (rc, msg)
    rc, msg = _create(lib, _bad(lambda p: permute_row(p, False)), ws=257)
    assert rc == hprlp.EINVAL and "workspace" in msg, (rc, msg)


def test_null_out_pointer(lib):
    o = hprlp.default_options()
    rc = lib.hprlp_create(None, 1, 0, 1, None, None, None, None, None, None, None, C.byref(o),
                          None, 0, None)
    assert rc == hprlp.EINVAL


def _create_batched(lib, lp, row_off, col_off, m1s, lams=None, ws=257, **opt):
    # ws is a misaligned fake pointer: a case that wrongly passed validation would stop at
    # the workspace check instead of reaching the GPU
    o = hprlp.default_options(**opt)
    arrs = [np.ascontiguousarray(lp.rowptr, dtype=np.int64),
            np.ascontiguousarray(lp.colidx, dtype=np.int32)] + \
        [np.ascontiguousarray(a, dtype=np.float64) for a in (lp.val, lp.b, lp.c, lp.l, lp.u)]
    inst = [np.ascontiguousarray(a, dtype=np.int64) for a in (row_off, col_off, m1s)]
    lam = None if lams is None else np.ascontiguousarray(lams, dtype=np.float64)
    h = C.c_void_p()
    rc = lib.hprlp_create_batched(C.byref(h), len(m1s), *[C.c_void_p(a.ctypes.data) for a in inst],
                                  *[C.c_void_p(a.ctypes.data) for a in arrs],
                                  None if lam is None else C.c_void_p(lam.ctypes.data),
                                  C.byref(o), C.c_void_p(ws), 1 << 30, None)
    return rc, lib.hprlp_last_error(None).decode()


def _two_instances():
    a = lpgen.bernoulli_lp(10, 10, 40, 0.2, seed=3)
    b = lpgen.bernoulli_lp(5, 15, 30, 0.2, seed=4)
    return lpgen.pack_block_diagonal([a, b])


@pytest.mark.parametrize("case,code", [
    ("offsets_do_not_start_at_0", hprlp.EDIM),
    ("offsets_not_increasing", hprlp.EDIM),
    ("m1_too_large", hprlp.EDIM),
    ("row_crosses_instances", hprlp.EDIM),
    ("check_every_one", hprlp.EINVAL),
    ("bad_lambda", hprlp.EINVAL),
    ("no_instances", hprlp.EDIM),
])
def test_create_batched_rejects_bad_layout(lib, case, code):
    lp = _two_instances()
    ro, co, m1s = lp.inst_row_off.copy(), lp.inst_col_off.copy(), lp.inst_m1.copy()
    opt, lams = {}, None
    if case == "offsets_do_not_start_at_0":
        ro[0] = 1
    elif case == "offsets_not_increasing":
        co[1] = 0
    elif case == "m1_too_large":
        m1s[0] = ro[1] - ro[0] + 1
    elif case == "row_crosses_instances":
        # move the first nonzero of instance 1 into instance 0's columns
        lp.colidx[lp.rowptr[ro[1]]] = 0
        lp.colidx[lp.rowptr[ro[1]]:lp.rowptr[ro[1] + 1]].sort()
        if len(set(lp.colidx[lp.rowptr[ro[1]]:lp.rowptr[ro[1] + 1]])) < \
                lp.rowptr[ro[1] + 1] - lp.rowptr[ro[1]]:
            pytest.skip("row became a repeat")
    elif case == "check_every_one":
        opt = dict(check_every=1)
    elif case == "bad_lambda":
        lams = [1.0, -2.0]
    else:
        m1s = m1s[:0]
    rc, msg = _create_batched(lib, lp, ro, co, m1s, lams, **opt)
    assert rc == code, (rc, msg)
    assert msg and "workspace" not in msg


def test_workspace_bytes_batched(lib):
    o = hprlp.default_options()
    a = hprlp.workspace_bytes_batched(4, 400, 800, 4000, o)
    assert a > hprlp.workspace_bytes(200, 200, 800, 4000, o)  # per-instance arrays on top
    with pytest.raises(hprlp.HPRLPError) as e:
        hprlp.workspace_bytes_batched(500, 400, 800, 4000, o)  # more instances than rows
    assert e.value.code == hprlp.EDIM


def test_workspace_covers_autotuner_candidates(lib):
    o = hprlp.default_options(chunk_nnz=8192, split_len=16384)
    ot = hprlp.default_options(chunk_nnz=8192, split_len=16384, autotune=1)
    assert hprlp.workspace_bytes(5000, 5000, 20000, 10**7, ot) > \
        hprlp.workspace_bytes(5000, 5000, 20000, 10**7, o)


def test_step_rejects_null_handle(lib):
    assert lib.hprlp_step(None, 10) == hprlp.EINVAL
    assert lib.hprlp_last_error(None)


def test_rho_out_of_range_is_rejected(lib):
    lp = lpgen.make("tiny")
    for rho in (-1.0, 2.5):
        rc, msg = _create(lib, lp, rho=rho)
        assert rc == hprlp.EINVAL, (rho, rc, msg)


def test_device_setup_scratch_is_in_the_workspace(lib):
    # the device preprocessing works inside the caller's workspace: at least 32 bytes per
    # nonzero more than the host preprocessing needs (sort buffers and the values as given)
    nnz = 10**6
    dev = hprlp.workspace_bytes(5000, 5000, 20000, nnz, hprlp.default_options())
    host = hprlp.workspace_bytes(5000, 5000, 20000, nnz, hprlp.default_options(setup_on_host=1))
    assert dev - host >= 32 * nnz
    mixed = hprlp.workspace_bytes(5000, 5000, 20000, nnz,
                                  hprlp.default_options(precision=hprlp.MIXED))
    mixed_host = hprlp.workspace_bytes(5000, 5000, 20000, nnz,
                                       hprlp.default_options(precision=hprlp.MIXED,
                                                             setup_on_host=1))
    assert mixed - mixed_host >= 48 * nnz


def test_t1_zero_limits(lib):
    o = hprlp.default_options(t1_zero=1)
    # G of 128 x 128 (m = 100 padded to the 64-wide panels) plus two 128 x 64 panels
    assert hprlp.workspace_bytes(100, 0, 400, 2000, o) >= hprlp.workspace_bytes(
        100, 0, 400, 2000, hprlp.default_options()) + 8 * (128 * 128 + 2 * 128 * 64)
    with pytest.raises(hprlp.HPRLPError) as e:
        hprlp.workspace_bytes(100, 5, 400, 2000, o)  # inequality rows
    assert e.value.code == hprlp.EINVAL
    with pytest.raises(hprlp.HPRLPError) as e:
        hprlp.workspace_bytes(65537, 0, 400000, 2000000, o)  # beyond the dense inverse
    assert e.value.code == hprlp.EDIM
    assert hprlp.workspace_bytes(65536, 0, 400000, 2000000, o) >= 8 * 65536 * 65536
    assert hprlp.workspace_bytes(8193, 0, 40000, 200000, o) >= 8 * 8256 * 8256
    with pytest.raises(hprlp.HPRLPError) as e:
        hprlp.workspace_bytes(100, 0, 400, 2000, hprlp.default_options(t1_zero=1,
                                                                       precision=hprlp.MIXED))
    assert e.value.code == hprlp.EINVAL
    with pytest.raises(hprlp.HPRLPError) as e:
        hprlp.workspace_bytes_batched(2, 100, 400, 2000, o)
    assert e.value.code == hprlp.EINVAL
    with pytest.raises(hprlp.HPRLPError):
        hprlp.workspace_bytes(100, 0, 400, 2000, hprlp.default_options(t1_zero=2))


def test_create_rejects_a_workspace_sized_for_host_preprocessing(lib):
    # the default (device) preprocessing needs its scratch inside the workspace: a workspace
    # sized with setup_on_host = 1 is rejected before any HIP call, naming the size it needs
    lp = lpgen.make("tiny")
    small = hprlp.workspace_bytes(lp.m1, lp.m2, lp.n, lp.nnz,
                                  hprlp.default_options(setup_on_host=1))
    need = hprlp.workspace_bytes(lp.m1, lp.m2, lp.n, lp.nnz, hprlp.default_options())
    assert small < need
    o = hprlp.default_options()
    arrs = [np.ascontiguousarray(lp.rowptr, dtype=np.int64),
            np.ascontiguousarray(lp.colidx, dtype=np.int32)] + \
        [np.ascontiguousarray(a, dtype=np.float64) for a in (lp.val, lp.b, lp.c, lp.l, lp.u)]
    h = C.c_void_p()
    rc = lib.hprlp_create(C.byref(h), lp.m1, lp.m2, lp.n, *[C.c_void_p(a.ctypes.data) for a in arrs],
                          C.byref(o), C.c_void_p(256), small, None)
    msg = lib.hprlp_last_error(None).decode()
    assert rc == hprlp.EINVAL and "workspace too small" in msg and str(need) in msg, msg


def test_tile_order_option(lib):
    # 0 (default, row order), 1 and -1 (the autotuner decides) are the values; column order
    # needs the row-order slot of every nonzero in the workspace (2 bytes per nonzero per
    # matrix) when it may be used, and is refused with T1 = 0, whose kernels read A row by row
    assert hprlp.default_options().tile_order == 0
    nnz = 10**6
    base = hprlp.workspace_bytes(5000, 5000, 20000, nnz, hprlp.default_options(tile_order=0))
    forced = hprlp.workspace_bytes(5000, 5000, 20000, nnz, hprlp.default_options(tile_order=1))
    tuned = hprlp.workspace_bytes(5000, 5000, 20000, nnz,
                                  hprlp.default_options(tile_order=-1, autotune=1))
    untuned = hprlp.workspace_bytes(5000, 5000, 20000, nnz, hprlp.default_options(tile_order=-1))
    assert forced - base >= 4 * nnz and untuned == base
    assert tuned - hprlp.workspace_bytes(5000, 5000, 20000, nnz,
                                         hprlp.default_options(tile_order=0, autotune=1)) >= 4 * nnz
    for bad in (dict(tile_order=2), dict(tile_order=-2), dict(tile_order=1, t1_zero=1)):
        with pytest.raises(hprlp.HPRLPError) as e:
            hprlp.workspace_bytes(100, 0, 400, 2000, hprlp.default_options(**bad))
        assert e.value.code == hprlp.EINVAL, bad
    # T1 = 0 with -1: row order, no slots
    t1 = hprlp.default_options(t1_zero=1, autotune=1, tile_order=-1)
    assert hprlp.workspace_bytes(100, 0, 400, 2000, t1) == hprlp.workspace_bytes(
        100, 0, 400, 2000, hprlp.default_options(t1_zero=1, autotune=1, tile_order=0))


def test_bundle_rows_option(lib):
    # -1 (default: shift-structured runs of A), 0 and 1 (every equal-length run of A and A^T)
    # are the values; when bundles may be used, the workspace holds a bounded worst case of
    # their work items, partial-sum slots and one bundle's staging copy; refused with T1 = 0
    assert hprlp.default_options().bundle_rows == -1
    nnz = 10**6
    off = hprlp.workspace_bytes(5000, 5000, 20000, nnz, hprlp.default_options(bundle_rows=0))
    auto = hprlp.workspace_bytes(5000, 5000, 20000, nnz, hprlp.default_options())
    forced = hprlp.workspace_bytes(5000, 5000, 20000, nnz, hprlp.default_options(bundle_rows=1))
    assert auto == forced and auto - off >= 12 * nnz
    for bad in (dict(bundle_rows=2), dict(bundle_rows=-2), dict(bundle_rows=1, t1_zero=1)):
        with pytest.raises(hprlp.HPRLPError) as e:
            hprlp.workspace_bytes(100, 0, 400, 2000, hprlp.default_options(**bad))
        assert e.value.code == hprlp.EINVAL, bad
    # T1 = 0 with -1: bundles of A possible (the residual pass runs on the pass kernel)
    assert hprlp.workspace_bytes(1000, 0, 4000, 20000, hprlp.default_options(t1_zero=1)) > \
        hprlp.workspace_bytes(1000, 0, 4000, 20000, hprlp.default_options(t1_zero=1, bundle_rows=0))
