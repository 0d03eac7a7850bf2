"""GPU: FP32 storage of A (scaling folded into the passes) and the FP32 -> FP64 mixed mode,
against the FP64 oracle.

  * FP64_A32 (A in FP32, exact; FP64 vectors): same bar as the FP64 path, 100-iteration
    iterate parity <= 1e-10 (the products are exact in FP64, only summation order differs).
  * MIXED: FP32 vectors until rel. KKT <= 1e-5, then FP64.  Full solves must reach rel. KKT
    <= 1e-8 and agree with the oracle's objective to 1e-7 relative; the error of each result
    against the oracle is printed.
"""
import numpy as np
import pytest

import lpgen
import oracle
from paper_2408_12179_amd import hprlp

pytestmark = pytest.mark.gpu
STRESS = dict(tile_nnz=256, tile_rows=64, short_max=16, split_len=64, chunk_nnz=256)


def rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300)


@pytest.mark.parametrize("name,scale", [("tiny", 1), ("zipf1m", 0.004), ("transport10m", 0.01)])
@pytest.mark.parametrize("sched", [{}, STRESS], ids=["default", "stress"])
def test_a32_iterate_parity_100(name, scale, sched):
    lp = lpgen.make(name, scale)
    ref = oracle.solve(lp, max_iter=100)
    s = hprlp.Solver(lp, max_iter=100, lambda_override=ref.lam, precision=hprlp.FP64_A32,
                     **sched)
    sol = s.solve()
    errs = dict(x_cur=rel(s.iterate(hprlp.XCUR), ref.x_cur),
                y_cur=rel(s.iterate(hprlp.YCUR), ref.y_cur),
                x_bar=rel(sol.x, ref.x), y_bar=rel(sol.y, ref.y), z_bar=rel(sol.z, ref.z))
    print(name, scale, sched, {k: f"{v:.2e}" for k, v in errs.items()})
    for k, v in errs.items():
        assert v <= 1e-10, (k, v)


def test_a32_power_method_lambda():
    lp = lpgen.make("zipf1m", 0.004)
    ref = oracle.solve(lp, max_iter=1)
    s = hprlp.Solver(lp, max_iter=1, precision=hprlp.FP64_A32)
    s.solve()
    assert abs(s.stats()["lambda"] - ref.lam) <= 1e-9 * ref.lam


@pytest.mark.parametrize("name,scale", [("tiny", 1), ("zipf1m", 0.0005), ("transport10m", 0.02), ("batch256", 0.004)])
def test_mixed_full_solve_against_oracle(name, scale):
    lp = lpgen.make(name, scale)
    if lp.inst_m1 is not None:
        lp = lp.instance(0)
    ref = oracle.solve(lp, max_iter=300000)
    assert ref.status == "OPTIMAL"
    s = hprlp.Solver(lp, precision=hprlp.MIXED, max_iter=300000)
    sol = s.solve()
    st = sol.stats
    err = abs(st["pobj"] - ref.pobj) / (1 + abs(ref.pobj))
    print(f"{name} mixed: {st['iters']} it ({st['iters_fp32']} FP32) vs oracle {ref.iters}; "
          f"obj err vs oracle {err:.2e}; x err {rel(sol.x, ref.x):.2e}")
    assert sol.status == "OPTIMAL"
    assert max(st["rel_p"], st["rel_d"], st["rel_gap"]) <= 1e-8
    assert st["iters_fp32"] > 0
    assert err <= 1e-7
    from lp_truth import relative_kkt
    assert max(relative_kkt(lp, sol.x, sol.y, sol.z)) <= 1.5e-8


def test_mixed_fp32_phase_tracks_oracle():
    # 100 FP32 iterations stay close to the FP64 iterates (FP32 rounding only)
    lp = lpgen.make("tiny")
    ref = oracle.solve(lp, max_iter=100)
    s = hprlp.Solver(lp, max_iter=100, lambda_override=ref.lam, precision=hprlp.MIXED)
    s.solve()
    assert rel(s.iterate(hprlp.XCUR), ref.x_cur) <= 1e-4
    assert rel(s.iterate(hprlp.YCUR), ref.y_cur) <= 1e-4
