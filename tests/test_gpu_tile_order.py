"""Column-ordered tiles (tile_order = 1) against row order (tile_order = 0), on the GPU.

Inside a tile the nonzeros are stored in column order and each product is staged at its
row-order slot before the row sums, so every sum is formed in the same order as in row
order: the two solves must agree bit for bit (w_bar, the current iterate, the check trace,
iteration and restart counts), for single LPs and batches (with instances stopping and the
schedules compacted), in FP64, FP64_A32 and MIXED, under the default and a stress schedule
(short tiles, whole-workgroup rows and split rows, which keep row order).  hprlp_get_schedule
reports the order in use.
"""
import numpy as np
import pytest

import lpgen
from paper_2408_12179_amd import hprlp

pytestmark = pytest.mark.gpu
STRESS = dict(tile_nnz=256, tile_rows=64, short_max=16, split_len=64, chunk_nnz=256)
PRECS = {"fp64": hprlp.FP64, "fp64a32": hprlp.FP64_A32, "mixed": hprlp.MIXED}


def _run(lp, order, batched=False, **kw):
    s = hprlp.Solver(lp, batched=batched, tile_order=order, **kw)
    sol = s.solve()
    out = dict(x=sol.x, y=sol.y, z=sol.z, status=sol.status, iters=sol.stats["iters"],
               restarts=sol.stats["restarts"], fp32=sol.stats["iters_fp32"],
               order=(s.schedule(0)["column_order"], s.schedule(1)["column_order"]))
    if batched:
        out["inst"] = [(s.stats_instance(i)["iters"], s.stats_instance(i)["status"])
                       for i in range(len(lp.inst_m1))]
        out["trace"] = np.concatenate([s.trace_instance(i) for i in range(len(lp.inst_m1))])
    else:
        out["trace"] = s.trace()
        out["xcur"] = s.iterate(hprlp.XCUR)
        out["ycur"] = s.iterate(hprlp.YCUR)
    s.close()
    return out


def _same(a, b):
    assert b["order"] == (True, True) and a["order"] == (False, False)
    for k in a:
        if k == "order":
            continue
        if isinstance(a[k], np.ndarray):
            np.testing.assert_array_equal(a[k], b[k], err_msg=k)
        else:
            assert a[k] == b[k], k


@pytest.mark.parametrize("prec", list(PRECS))
@pytest.mark.parametrize("sched", [{}, STRESS], ids=["default", "stress"])
@pytest.mark.parametrize("name,scale", [("zipf1m", 0.004), ("transport10m", 0.01)])
def test_single_lp_bitwise(name, scale, sched, prec):
    lp = lpgen.make(name, scale)
    kw = dict(max_iter=2000, precision=PRECS[prec], **sched)
    _same(_run(lp, 0, **kw), _run(lp, 1, **kw))


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batched_bitwise_with_compaction(prec):
    lp = lpgen.batched_lp(8, m_range=(60, 400), name="full8")
    kw = dict(check_every=100, precision=PRECS[prec], max_iter=200000)
    a, b = _run(lp, 0, batched=True, **kw), _run(lp, 1, batched=True, **kw)
    assert a["status"] == "OPTIMAL"
    _same(a, b)
