"""GPU parity of batched solves: n LPs packed block-diagonally and solved in one run (one
hipGraph per check_every-iteration chunk, per-instance decisions on the device), each
instance against the FP64 CPU oracle solving that instance alone.

Bars as for single LPs: iterates <= 1e-10 relative after a fixed number of iterations (lambda
taken from the oracle so both run the same map), identical check-level decisions (iteration
of termination, restart count), and for full solves rel. KKT <= 1e-8 with objectives within
1e-7 relative of the oracle's.
"""
import numpy as np
import pytest

import lpgen
import oracle
from paper_2408_12179_amd import hprlp

pytestmark = pytest.mark.gpu

STRESS = dict(tile_nnz=256, tile_rows=64, short_max=16, split_len=64, chunk_nnz=256)
CE = 100  # check period of the batched workload


def rel(a, b):
    d = np.linalg.norm(a - b)
    nb = np.linalg.norm(b)
    return d / nb if nb > 0 else d


def hetero_batch():
    """Instances of different shapes: equality-only, inequality-only, ragged Zipf rows with
    long rows, free variables, a single row, and plain Bernoulli ones."""
    parts = [lpgen.bernoulli_lp(40, 0, 90, 0.08, seed=11),
             lpgen.bernoulli_lp(0, 40, 90, 0.08, seed=12),
             lpgen.zipf_lp(117, 89, 411, seed=16, row_len=(1, 70)),
             lpgen.zipf_lp(30, 30, 120, seed=15, free_frac=1.0),
             lpgen.bernoulli_lp(1, 0, 30, 0.5, seed=14),
             lpgen.bernoulli_lp(25, 25, 100, 0.06, seed=17)]
    return lpgen.pack_block_diagonal(parts, "hetero")


def small_batch(n_inst=7):
    return lpgen.batched_lp(n_inst, m_range=(20, 120), name="small")


def _instance_outputs(sol, lp, i):
    r0, r1 = lp.inst_row_off[i], lp.inst_row_off[i + 1]
    c0, c1 = lp.inst_col_off[i], lp.inst_col_off[i + 1]
    return sol.x[c0:c1], sol.y[r0:r1], sol.z[c0:c1]


def _batched_iterate_parity(lp, iters, **sched):
    n_inst = len(lp.inst_m1)
    refs = [oracle.solve(lp.instance(i), max_iter=iters, check_every=CE) for i in range(n_inst)]
    lams = [r.lam for r in refs]
    s = hprlp.Solver(lp, batched=True, lambdas=lams, max_iter=iters, check_every=CE, **sched)
    sol = s.solve()
    worst = 0.0
    for i, ref in enumerate(refs):
        st = s.stats_instance(i)
        assert st["iters"] == ref.iters, (i, st["iters"], ref.iters)
        assert st["restarts"] == ref.restarts, (i, st["restarts"], ref.restarts)
        assert st["status"] == ref.status, (i, st["status"], ref.status)
        x, y, z = _instance_outputs(sol, lp, i)
        for name, a, b in (("x", x, ref.x), ("y", y, ref.y), ("z", z, ref.z)):
            e = rel(a, b)
            worst = max(worst, e)
            assert e <= 1e-10, (i, name, e)
        tr = s.trace_instance(i)
        assert len(tr) == min(len(ref.trace), 64)
        np.testing.assert_array_equal(tr[:, 0], ref.trace[:len(tr), 0])     # k
        np.testing.assert_array_equal(tr[:, 8], ref.trace[:len(tr), 16])    # restarted
        # sigma next (eq. sigma): a ratio of ||x_bar - x0|| and ||y_bar - y0||, which late in a
        # solve are ~1e-6 of ||x||, so the iterates' ~1e-15 rounding shows up as ~1e-9 here
        np.testing.assert_allclose(tr[:, 9], ref.trace[:len(tr), 17], rtol=1e-7)
    n_comp = sol.stats["n_compactions"]
    print(lp.name, n_inst, iters, sched, f"worst {worst:.2e}", "compactions", n_comp,
          "stopped", [s.stats_instance(i)["iters"] for i in range(n_inst)])
    s.close()
    return n_comp


@pytest.mark.parametrize("sched", [{}, STRESS], ids=["default", "stress"])
def test_batched_iterate_parity_small(sched):
    _batched_iterate_parity(small_batch(), 300, **sched)


@pytest.mark.parametrize("sched", [{}, STRESS], ids=["default", "stress"])
def test_batched_iterate_parity_heterogeneous(sched):
    _batched_iterate_parity(hetero_batch(), 400, **sched)


@pytest.mark.parametrize("sched", [{}, STRESS], ids=["default", "stress"])
def test_batched_parity_while_instances_stop(sched):
    # long enough for most instances to reach 1e-8 and stop: the schedules are rebuilt over
    # the instances still iterating, whose iterates must stay on the oracle's
    lp = lpgen.batched_lp(10, m_range=(20, 160), name="stop10")
    n = _batched_iterate_parity(lp, 3000, **sched)
    assert n >= 1


def test_batched_lambda_per_instance():
    lp = small_batch(5)
    s = hprlp.Solver(lp, batched=True, max_iter=CE, check_every=CE)
    s.solve()
    for i in range(5):
        ref = oracle.solve(lp.instance(i), max_iter=1)
        st = s.stats_instance(i)
        assert abs(st["lambda"] - ref.lam) <= 1e-9 * ref.lam, (i, st["lambda"], ref.lam)


def test_batched_full_solve_parity():
    lp = lpgen.batched_lp(8, m_range=(60, 400), name="full8")
    s = hprlp.Solver(lp, batched=True, check_every=CE)
    sol = s.solve()
    assert sol.status == "OPTIMAL"
    from lp_truth import relative_kkt
    for i in range(8):
        inst = lp.instance(i)
        ref = oracle.solve(inst, check_every=CE)
        st = s.stats_instance(i)
        assert ref.status == "OPTIMAL" and st["status"] == "OPTIMAL"
        assert max(st["rel_p"], st["rel_d"], st["rel_gap"]) <= 1e-8
        assert abs(st["pobj"] - ref.pobj) <= 1e-7 * (1 + abs(ref.pobj)), (i, st["pobj"], ref.pobj)
        assert abs(st["pobj"] - inst.cert.obj) <= 1e-7 * (1 + abs(inst.cert.obj))
        assert st["iters"] == ref.iters, (i, st["iters"], ref.iters)
        x, y, z = _instance_outputs(sol, lp, i)
        assert max(relative_kkt(inst, x, y, z)) <= 1.5e-8
    print("full8 iters", [s.stats_instance(i)["iters"] for i in range(8)],
          f"{sol.stats['t_solve_ms']:.1f} ms")


def test_batched_mixed_full_solve():
    lp = lpgen.batched_lp(8, m_range=(60, 400), name="full8")
    s = hprlp.Solver(lp, batched=True, check_every=CE, precision=hprlp.MIXED)
    sol = s.solve()
    assert sol.status == "OPTIMAL"
    assert sol.stats["iters_fp32"] > 0
    from lp_truth import relative_kkt
    for i in range(8):
        inst = lp.instance(i)
        st = s.stats_instance(i)
        assert max(st["rel_p"], st["rel_d"], st["rel_gap"]) <= 1e-8
        assert abs(st["pobj"] - inst.cert.obj) <= 1e-7 * (1 + abs(inst.cert.obj))
        x, y, z = _instance_outputs(sol, lp, i)
        assert max(relative_kkt(inst, x, y, z)) <= 1.5e-8


@pytest.mark.parametrize("prec", [hprlp.FP64_A32])
def test_batched_a32_iterate_parity(prec):
    lp = small_batch(4)
    iters = 200
    refs = [oracle.solve(lp.instance(i), max_iter=iters, check_every=CE) for i in range(4)]
    s = hprlp.Solver(lp, batched=True, lambdas=[r.lam for r in refs], max_iter=iters,
                     check_every=CE, precision=prec)
    sol = s.solve()
    for i, ref in enumerate(refs):
        x, y, z = _instance_outputs(sol, lp, i)
        assert rel(x, ref.x) <= 1e-10 and rel(y, ref.y) <= 1e-10, i


def test_batched_single_instance_matches_single_lp():
    # a batch of one is the single-LP solve with the same check period (same decisions)
    lp = lpgen.make("tiny")
    packed = lpgen.pack_block_diagonal([lp], "one")
    ref = oracle.solve(lp, max_iter=500, check_every=CE)
    a = hprlp.Solver(packed, batched=True, lambdas=[ref.lam], max_iter=500, check_every=CE,
                     reorder=0)
    sa = a.solve()
    b = hprlp.Solver(lp, lambda_override=ref.lam, max_iter=500, check_every=CE, reorder=0)
    sb = b.solve()
    assert rel(sa.x, sb.x) <= 1e-12 and rel(sa.y, sb.y) <= 1e-12
    assert rel(sa.x, ref.x) <= 1e-10


def test_batched_deterministic_and_resolvable():
    lp = small_batch(6)
    s = hprlp.Solver(lp, batched=True, max_iter=400, check_every=CE, **STRESS)
    a = s.solve()
    b = s.solve()  # the graphs are reused; state is re-initialised by every solve
    assert np.array_equal(a.x, b.x) and np.array_equal(a.y, b.y)
    assert a.stats["iters"] == b.stats["iters"]


def test_batched_many_small_instances():
    # more instances than the decision kernel's 1024 threads and more reduction workgroups:
    # every instance must stop where the oracle stops; a sample is compared element-wise
    lp = lpgen.batched_lp(1500, m_range=(4, 12), rho_range=(2.0, 4.0), name="many")
    n_inst = len(lp.inst_m1)
    s = hprlp.Solver(lp, batched=True, lambdas=np.ones(n_inst), max_iter=2000, check_every=CE)
    sol = s.solve()
    for i in (0, 1023, 1024, 1499):
        ref = oracle.solve(lp.instance(i), max_iter=2000, check_every=CE, lambda_override=1.0)
        st = s.stats_instance(i)
        assert st["iters"] == ref.iters and st["status"] == ref.status, (i, st["iters"], ref.iters)
        x, y, z = _instance_outputs(sol, lp, i)
        assert rel(x, ref.x) <= 1e-10 and rel(y, ref.y) <= 1e-10, i
    print("many: statuses", {k: sum(s.stats_instance(i)["status"] == k for i in range(n_inst))
                             for k in ("OPTIMAL", "ITER_LIMIT")}, "compactions",
          sol.stats["n_compactions"])


def test_begin_step_chunks_equal_solve_and_event_nodes():
    """hprlp_begin + hprlp_step(k * check_every) runs the same chunks as hprlp_solve: the
    same w_bar bit for bit, the same per-instance stops, restarts and statuses, and the
    check-level decisions still match the oracle.  profile = N places HIP event nodes in the
    chunk graphs; it must not change a bit of the iterates and must time every N-th
    iteration's passes."""
    lp = small_batch(5)
    n_inst = len(lp.inst_m1)
    iters = 3000
    refs = [oracle.solve(lp.instance(i), max_iter=iters, check_every=CE) for i in range(n_inst)]
    lams = [r.lam for r in refs]
    a = hprlp.Solver(lp, batched=True, lambdas=lams, max_iter=iters, check_every=CE)
    sa = a.solve()
    for prof in (0, 10):
        b = hprlp.Solver(lp, batched=True, lambdas=lams, max_iter=iters, check_every=CE,
                         profile=prof)
        st0 = b.begin()
        assert st0["iters"] == 0
        for _ in range(iters // (3 * CE)):
            b.step(3 * CE)
        st = b.stats()
        assert st["iters"] <= iters
        x, y, z = (b.iterate(w) for w in (hprlp.XBAR, hprlp.YBAR, hprlp.ZBAR))
        np.testing.assert_array_equal(x, sa.x)
        np.testing.assert_array_equal(y, sa.y)
        np.testing.assert_array_equal(z, sa.z)
        for i, ref in enumerate(refs):
            si = b.stats_instance(i)
            assert si["iters"] == ref.iters and si["restarts"] == ref.restarts, i
            assert si["status"] == ref.status, i
            assert 0 < si["t_solve_ms"] <= st["t_solve_ms"] + 1e-9
        if prof:
            chunks = st["iters"] // CE
            assert st["col_pass_launches"] == st["row_pass_launches"] == chunks * (CE // prof)
            assert st["col_pass_ms"] > 0 and st["row_pass_ms"] > 0
        else:
            assert st["col_pass_launches"] == 0
        with pytest.raises(hprlp.HPRLPError):
            b.step(CE + 1)  # a batch steps in whole chunks
        b.close()
    a.close()
