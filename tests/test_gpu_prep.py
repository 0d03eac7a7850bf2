"""Device preprocessing (the default) against the host preprocessing (setup_on_host = 1).

The two paths compute the same column order, transpose, scaling (Section 4.1) and data
vectors in the same order of operations, so everything downstream must agree bit for bit:
D_r, D_c, the schedules, and the iterates after a few hundred iterations, across restarts
and sigma updates.  The cases cover the renumbering on and off, the three precisions,
batches, Ruiz / Pock-Chambolle switched off, empty rows and columns, a single row, one
column, many empty columns, rows long enough to be split, and inputs spanning many radix
sort tiles."""
import numpy as np
import pytest

import lpgen
from paper_2408_12179_amd import hprlp

pytestmark = pytest.mark.gpu


def _drop(lp, keep):
    """Remove the nonzeros where keep is False (row structure kept)."""
    row_of = np.repeat(np.arange(lp.m), np.diff(lp.rowptr))
    lens = np.bincount(row_of[keep], minlength=lp.m)
    lp.rowptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    lp.colidx, lp.val = lp.colidx[keep], lp.val[keep]
    return lp


def _case(name):
    if name == "empty_row_and_col":
        lp = lpgen.bernoulli_lp(30, 30, 100, 0.06, seed=13)
        keep = np.ones(lp.nnz, dtype=bool)
        keep[lp.rowptr[0]:lp.rowptr[1]] = False
        keep[lp.rowptr[30]:lp.rowptr[31]] = False
        keep &= lp.colidx != 0
        lp = _drop(lp, keep)
        lp.b[0], lp.b[30] = 0.0, -1.0
        return lp, {}
    if name == "many_empty_columns":  # n far above the columns that hold a nonzero
        lp = lpgen.zipf_lp(200, 100, 6000, seed=21, row_len=(1, 12))
        return lp, {}
    if name == "single_row":
        return lpgen.bernoulli_lp(1, 0, 30, 0.5, seed=14), {}
    if name == "one_column":
        lp = lpgen.LP("one_column", 1, 2, 1, np.array([0, 1, 2, 3], dtype=np.int64),
                      np.zeros(3, dtype=np.int32), np.array([2.0, 1.0, -1.0]),
                      np.array([2.0, 0.5, -3.0]), np.array([1.0]), np.array([0.0]),
                      np.array([4.0]))
        return lp, {}
    if name == "long_rows_split":  # rows and columns beyond split_len: chunked items
        lp = lpgen.zipf_lp(300, 200, 900, seed=22, row_len=(1, 400))
        return lp, dict(tile_nnz=256, tile_rows=64, short_max=16, split_len=64, chunk_nnz=256)
    if name == "no_ruiz_no_pc":
        return lpgen.make("zipf1m", 0.004), dict(ruiz_iters=0, pock_chambolle=0)
    if name == "pc_only":
        return lpgen.make("zipf1m", 0.004), dict(ruiz_iters=0)
    if name == "no_reorder":
        return lpgen.make("zipf1m", 0.004), dict(reorder=0)
    if name == "transport":
        return lpgen.make("transport10m", 0.002), {}
    if name == "zipf_mixed":
        return lpgen.make("zipf1m", 0.004), dict(precision=hprlp.MIXED)
    if name == "zipf_a32":
        return lpgen.make("zipf1m", 0.004), dict(precision=hprlp.FP64_A32)
    if name == "zipf_many_tiles":  # ~180k nonzeros: 44 sort tiles
        return lpgen.make("zipf1m", 0.016), {}
    if name == "t1_zero":  # the dense inverse of A~A~^T built from either path's arrays
        return lpgen.ot_lp(20, 30, seed=501), dict(t1_zero=1)
    return lpgen.make(name), {}


CASES = ["tiny", "empty_row_and_col", "many_empty_columns", "single_row", "one_column",
         "long_rows_split", "no_ruiz_no_pc", "pc_only", "no_reorder", "transport",
         "zipf_mixed", "zipf_a32", "zipf_many_tiles", "t1_zero"]


def _pair(lp, iters, batched=False, lambdas=None, **opt):
    out = []
    for host in (1, 0):
        s = hprlp.Solver(lp, batched=batched, lambdas=lambdas, max_iter=iters,
                         setup_on_host=host, **opt)
        sol = s.solve()
        r = dict(x=sol.x, y=sol.y, z=sol.z, stats=sol.stats,
                 dr=s.iterate(hprlp.DROW) if not batched else None,
                 dc=s.iterate(hprlp.DCOL) if not batched else None,
                 schedA=s.schedule(0), schedT=s.schedule(1))
        if not batched:
            r["xcur"] = s.iterate(hprlp.XCUR)
            r["ycur"] = s.iterate(hprlp.YCUR)
        s.close()
        out.append(r)
    return out


def _same(a, b, what):
    assert a.shape == b.shape and np.array_equal(a.view(np.uint64), b.view(np.uint64)), \
        (what, np.max(np.abs(a - b)))


@pytest.mark.parametrize("case", CASES)
def test_device_setup_bitwise(case):
    lp, opt = _case(case)
    h, d = _pair(lp, 400, **opt)  # lambda from the power method on each side
    for k in ("dr", "dc", "x", "y", "z", "xcur", "ycur"):
        _same(d[k], h[k], (case, k))
    assert d["schedA"] == h["schedA"] and d["schedT"] == h["schedT"]
    for k in ("iters", "restarts", "power_iters", "lambda", "sigma", "pobj", "rel_p", "rel_d",
              "beta_b", "beta_c"):
        _same(np.float64(d["stats"][k]), np.float64(h["stats"][k]), (case, k))
    print(case, lp.m, lp.n, lp.nnz, "prep ms host/device",
          round(h["stats"]["t_prep_ms"], 2), round(d["stats"]["t_prep_ms"], 2))


def test_device_setup_with_power_method_and_full_solve():
    lp = lpgen.make("tiny")
    h, d = _pair(lp, 10**6)
    assert d["stats"]["status"] == "OPTIMAL" and d["stats"]["lambda"] == h["stats"]["lambda"]
    for k in ("x", "y", "z"):
        _same(d[k], h[k], k)


@pytest.mark.parametrize("prec", [hprlp.FP64, hprlp.MIXED])
def test_device_setup_batched(prec):
    lp = lpgen.batched_lp(6, m_range=(40, 600), name="prep6")
    ni = len(lp.inst_m1)
    h, d = _pair(lp, 300, batched=True, lambdas=np.ones(ni), check_every=50, precision=prec)
    for k in ("x", "y", "z"):
        _same(d[k], h[k], k)
    assert d["schedA"] == h["schedA"] and d["schedT"] == h["schedT"]
    assert d["stats"]["iters"] == h["stats"]["iters"]
