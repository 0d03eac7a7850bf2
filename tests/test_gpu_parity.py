"""GPU parity: the HIP path (through the C ABI) against the FP64 CPU oracle on the same
seeded inputs.

Bars (the termination test of Section 4.1 is rel. KKT <= 1e-8; the iterate bar leaves room
for different summation orders, about 1e-16 per operation, through a nonexpansive map):
  * iterates after 100 iterations: norm-wise relative difference <= 1e-10
    (lambda taken from the oracle so both run the same map; scaling is compared separately);
  * full solves: both reach relative KKT <= 1e-8 and the objectives agree to 1e-7 relative;
  * preconditioning: D_r, D_c agree to 1e-14 relative; lambda (power method) to 1e-9.
"""
import numpy as np
import pytest

import lpgen
import oracle
from paper_2408_12179_amd import hprlp

pytestmark = pytest.mark.gpu

# a schedule that forces every work-item kind (tiles, whole-workgroup rows, split rows) even
# on small matrices
STRESS = dict(tile_nnz=256, tile_rows=64, short_max=16, split_len=64, chunk_nnz=256)


def rel(a, b):
    d = np.linalg.norm(a - b)
    nb = np.linalg.norm(b)
    return d / nb if nb > 0 else d


def _iterate_parity(lp, iters=100, **sched):
    ref = oracle.solve(lp, max_iter=iters)
    s = hprlp.Solver(lp, max_iter=iters, lambda_override=ref.lam, **sched)
    sol = s.solve()
    assert sol.status in ("ITER_LIMIT", "OPTIMAL")
    assert sol.stats["iters"] == ref.iters
    out = dict(x_cur=rel(s.iterate(hprlp.XCUR), ref.x_cur),
               y_cur=rel(s.iterate(hprlp.YCUR), ref.y_cur),
               x_bar=rel(sol.x, ref.x), y_bar=rel(sol.y, ref.y), z_bar=rel(sol.z, ref.z))
    print(lp.name, iters, sched, {k: f"{v:.2e}" for k, v in out.items()})
    for k, v in out.items():
        assert v <= 1e-10, (k, v)
    # scaling: same definition, same order of operations
    assert rel(s.iterate(hprlp.DROW), ref.dr) <= 1e-14
    assert rel(s.iterate(hprlp.DCOL), ref.dc) <= 1e-14
    s.close()


@pytest.mark.parametrize("sched", [{}, STRESS], ids=["default", "stress"])
def test_tiny_iterate_parity_100(sched):
    _iterate_parity(lpgen.make("tiny"), **sched)


@pytest.mark.parametrize("name,scale", [("zipf1m", 0.004), ("transport10m", 0.01)])
@pytest.mark.parametrize("sched", [{}, STRESS], ids=["default", "stress"])
def test_downscaled_iterate_parity(name, scale, sched):
    _iterate_parity(lpgen.make(name, scale), **sched)


def test_iterate_parity_across_restarts():
    # 700 iterations: several checks, restarts and sigma updates on both sides
    lp = lpgen.make("tiny")
    ref = oracle.solve(lp, max_iter=700)
    s = hprlp.Solver(lp, max_iter=700, lambda_override=ref.lam)
    sol = s.solve()
    tr = s.trace()
    assert len(tr) == len(ref.trace)
    np.testing.assert_array_equal(tr[:, 0], ref.trace[:, 0])        # k
    np.testing.assert_array_equal(tr[:, 16], ref.trace[:, 16])      # restart decisions
    np.testing.assert_allclose(tr[:, 3], ref.trace[:, 3], rtol=1e-9)  # sigma
    np.testing.assert_allclose(tr[:, 4], ref.trace[:, 4], rtol=1e-8)  # merit
    np.testing.assert_allclose(tr[:, 7:10], ref.trace[:, 7:10], rtol=1e-6, atol=1e-14)
    assert rel(s.iterate(hprlp.XCUR), ref.x_cur) <= 1e-9
    assert rel(s.iterate(hprlp.YCUR), ref.y_cur) <= 1e-9


def test_power_method_lambda():
    lp = lpgen.make("tiny")
    ref = oracle.solve(lp, max_iter=1)
    s = hprlp.Solver(lp, max_iter=1)
    s.solve()
    st = s.stats()
    assert abs(st["lambda"] - ref.lam) <= 1e-9 * ref.lam
    assert abs(st["power_iters"] - ref.power_iters) <= 2


def test_tiny_full_solve_parity():
    lp = lpgen.make("tiny")
    ref = oracle.solve(lp)
    s = hprlp.Solver(lp)
    sol = s.solve()
    st = sol.stats
    print("tiny full", st["iters"], ref.iters, st["pobj"], ref.pobj, st["t_solve_ms"])
    assert ref.status == "OPTIMAL" and sol.status == "OPTIMAL"
    assert max(st["rel_p"], st["rel_d"], st["rel_gap"]) <= 1e-8
    assert abs(st["pobj"] - ref.pobj) <= 1e-7 * (1 + abs(ref.pobj))
    assert abs(st["pobj"] - lp.cert.obj) <= 1e-7 * (1 + abs(lp.cert.obj))
    # the returned point, re-evaluated independently of both solvers
    from lp_truth import relative_kkt
    assert max(relative_kkt(lp, sol.x, sol.y, sol.z)) <= 1.5e-8


def test_deterministic_bitwise():
    lp = lpgen.make("zipf1m", 0.004)
    a = hprlp.Solver(lp, max_iter=600, **STRESS)
    sa = a.solve()
    b = hprlp.Solver(lp, max_iter=600, **STRESS)
    sb = b.solve()
    assert np.array_equal(sa.x, sb.x) and np.array_equal(sa.y, sb.y)
    assert np.array_equal(a.trace(), b.trace())


def test_outputs_to_device_pointers():
    import torch
    lp = lpgen.make("tiny")
    s = hprlp.Solver(lp, max_iter=300)
    h = s.solve()
    x, y, z, st = s.solve_device()
    assert st == h.status
    assert np.array_equal(x.cpu().numpy(), h.x) and np.array_equal(y.cpu().numpy(), h.y)
    assert np.array_equal(z.cpu().numpy(), h.z)
    del torch


@pytest.mark.parametrize("case", ["m2_zero", "m1_zero", "empty_row_and_col", "single_row",
                                  "free_only", "ragged_tiles"])
def test_edge_cases_parity(case):
    rng = np.random.default_rng(7)
    if case == "m2_zero":
        lp = lpgen.bernoulli_lp(40, 0, 90, 0.08, seed=11)
    elif case == "m1_zero":
        lp = lpgen.bernoulli_lp(0, 40, 90, 0.08, seed=12)
    elif case == "empty_row_and_col":
        lp = lpgen.bernoulli_lp(30, 30, 100, 0.06, seed=13)
        # empty the first row of each block and zero out column 0
        rp, ci, va = lp.rowptr, lp.colidx, lp.val
        keep = np.ones(lp.nnz, dtype=bool)
        keep[rp[0]:rp[1]] = False
        keep[rp[30]:rp[31]] = False
        keep &= ci != 0
        row_of = np.repeat(np.arange(lp.m), np.diff(rp))
        lens = np.bincount(row_of[keep], minlength=lp.m)
        lp.rowptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        lp.colidx, lp.val = ci[keep], va[keep]
        lp.b[0], lp.b[30] = 0.0, -1.0  # consistent with an empty row (0 = 0, 0 >= -1)
    elif case == "single_row":
        lp = lpgen.bernoulli_lp(1, 0, 30, 0.5, seed=14)
    elif case == "free_only":
        lp = lpgen.zipf_lp(60, 60, 240, seed=15, free_frac=1.0)
    else:  # row count not a multiple of anything, tiles ending mid-stream
        lp = lpgen.zipf_lp(517, 389, 1811, seed=16, row_len=(1, 70))
    del rng
    ref = oracle.solve(lp, max_iter=100)
    for sched in ({}, STRESS):
        s = hprlp.Solver(lp, max_iter=100, lambda_override=ref.lam, **sched)
        sol = s.solve()
        assert rel(s.iterate(hprlp.XCUR), ref.x_cur) <= 1e-10, (case, sched)
        assert rel(s.iterate(hprlp.YCUR), ref.y_cur) <= 1e-10, (case, sched)
        assert rel(sol.x, ref.x) <= 1e-10 and rel(sol.y, ref.y) <= 1e-10
        s.close()


def test_step_continues_the_iteration():
    # 100 iterations (a check at the last one, no restart before k = 150), then 50 plain
    # iterations: the same current iterate as a 150-iteration solve and as the oracle's
    lp = lpgen.make("tiny")
    ref = oracle.solve(lp, max_iter=150)
    a = hprlp.Solver(lp, max_iter=100, lambda_override=ref.lam)
    a.solve()
    a.step(50)
    assert a.stats()["iters"] == 150
    b = hprlp.Solver(lp, max_iter=150, lambda_override=ref.lam)
    b.solve()
    for which, r in ((hprlp.XCUR, ref.x_cur), (hprlp.YCUR, ref.y_cur)):
        assert rel(a.iterate(which), b.iterate(which)) <= 1e-14
        assert rel(a.iterate(which), r) <= 1e-10
    assert b.stats()["t_setup_ms"] > 0


def test_infeasible_lp_runs_to_the_iteration_limit():
    # x1 + x2 = 3 with 0 <= x <= 1 has no feasible point and the method has no infeasibility
    # detection: both sides run to the limit with the same iterates and a large residual
    lp = lpgen.LP("infeasible", 1, 0, 2, np.array([0, 2], dtype=np.int64),
                  np.array([0, 1], dtype=np.int32), np.array([1.0, 1.0]), np.array([3.0]),
                  np.array([1.0, 2.0]), np.zeros(2), np.ones(2))
    ref = oracle.solve(lp, max_iter=3000)
    s = hprlp.Solver(lp, max_iter=3000, lambda_override=ref.lam)
    sol = s.solve()
    assert ref.status == sol.status == "ITER_LIMIT"
    assert sol.stats["rel_p"] > 1e-3 and np.all(np.isfinite(sol.x)) and np.all(np.isfinite(sol.y))
    assert rel(sol.x, ref.x) <= 1e-10


@pytest.mark.parametrize("name,scale,prec", [("tiny", 1, hprlp.FP64), ("zipf1m", 0.004, hprlp.FP64),
                                             ("transport10m", 0.01, hprlp.MIXED)])
def test_chunk_graphs_are_bitwise_identical(name, scale, prec):
    # plain iterations as captured graphs (device-resident scalars) against one launch per pass,
    # over several checks, restarts and (MIXED) the precision switch
    lp = lpgen.make(name, scale)
    kw = dict(max_iter=1000, precision=prec, lambda_override=0.9, stall_checks=2)
    a = hprlp.Solver(lp, graph=2, **kw)
    sa = a.solve()
    b = hprlp.Solver(lp, graph=0, **kw)
    sb = b.solve()
    assert np.array_equal(sa.x, sb.x) and np.array_equal(sa.y, sb.y) and np.array_equal(sa.z, sb.z)
    assert np.array_equal(a.iterate(hprlp.XCUR), b.iterate(hprlp.XCUR))
    assert np.array_equal(a.trace(), b.trace())
    assert sa.stats["restarts"] >= 1
