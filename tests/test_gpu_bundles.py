"""Row bundles (runs of equal-length long rows stored k-major, one lane per row) against the
oracle: the iterates after 100 iterations at the 1e-10 bar (norm-wise and entry by entry),
on the LPs where the default finds them (the demand rows of transportation and transport
LPs, whose columns shift by one from row to row) and with every equal-length run of A and
A^T bundled (dense LPs), in the three precisions, under a stress schedule, in a compacting
batch, at the edges of the bundle rules (minimum row length and bundle size, a run one row
longer than a bundle, inequality rows), full solves, and bitwise reproducibility."""
import numpy as np
import pytest

import lpgen
import oracle
from bundle_cases import dense, edge_lp, expected_shifted_bundles, ot, transport
from paper_2408_12179_amd import hprlp

pytestmark = pytest.mark.gpu

STRESS = dict(tile_nnz=256, tile_rows=64, short_max=16, split_len=64, chunk_nnz=256)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


def close_entrywise(a, b, tol=1e-10):
    scale = np.abs(b) + 1e-3 * (np.max(np.abs(b)) if b.size else 0.0)
    bad = (np.abs(a - b) > tol * scale) & ~((a == 0) & (b == 0))
    assert not bad.any(), (np.flatnonzero(bad)[:5], a[bad][:5], b[bad][:5])


def check(pairs, tol=1e-10):
    for name, a, b in pairs:
        assert rel(a, b) <= tol, (name, rel(a, b))
        close_entrywise(a, b, tol)


def iterates(s, sol, ref):
    return [("x_bar", sol.x, ref.x), ("y_bar", sol.y, ref.y), ("z_bar", sol.z, ref.z),
            ("x_cur", s.iterate(hprlp.XCUR), ref.x_cur), ("y_cur", s.iterate(hprlp.YCUR), ref.y_cur)]


@pytest.mark.parametrize("name", ["transport", "ot"])
def test_default_finds_shifted_rows(name):
    lp = {"transport": transport, "ot": ot}[name]()
    ref = oracle.solve(lp, max_iter=100)
    s = hprlp.Solver(lp, max_iter=100, lambda_override=ref.lam)
    sol = s.solve()
    sa, st = s.schedule(0), s.schedule(1)
    assert sa["bundle_items"] == expected_shifted_bundles(lp) > 0 and st["bundle_items"] == 0, \
        (sa, st)
    for w, got in ((0, sa), (1, st)):  # the schedule create built is the host plan's
        plan = hprlp.plan_schedule(lp, w)
        assert all(got[k] == plan[k] for k in plan), (w, got, plan)
    check(iterates(s, sol, ref))
    s.close()
    s0 = hprlp.Solver(lp, max_iter=100, lambda_override=ref.lam, bundle_rows=0)
    assert s0.schedule(0)["bundle_items"] == 0
    check(iterates(s0, s0.solve(), ref))
    s0.close()


def test_random_rows_are_not_bundled_by_default():
    lp = dense(n=300)
    s = hprlp.Solver(lp, max_iter=1)
    assert s.schedule(0)["bundle_items"] == 0 and s.schedule(1)["bundle_items"] == 0
    s.close()


@pytest.mark.parametrize("precision", [hprlp.FP64, hprlp.FP64_A32], ids=["fp64", "fp64a32"])
@pytest.mark.parametrize("sched", ["default", "stress"])
def test_forced_bundles_parity(precision, sched):
    lp = dense()
    ref = oracle.solve(lp, max_iter=100)
    extra = STRESS if sched == "stress" else {}
    s = hprlp.Solver(lp, max_iter=100, lambda_override=ref.lam, precision=precision,
                     bundle_rows=1, **extra)
    sol = s.solve()
    assert s.schedule(0)["bundle_items"] == 5 * 7   # 300 rows: 64 x 4 + 44; 400 = 6 * 64 + 16
    assert s.schedule(1)["bundle_items"] == 7 * 5   # 400 rows: 64 x 6 + 16; 300 = 4 * 64 + 44
    check(iterates(s, sol, ref))
    s.close()


def test_forced_bundles_power_method_and_checks():
    lp = dense(seed=604)
    ref = oracle.solve(lp, max_iter=300)
    s = hprlp.Solver(lp, max_iter=300, bundle_rows=1)
    sol = s.solve()
    assert abs(sol.stats["lambda"] - ref.lam) <= 1e-9 * ref.lam
    check(iterates(s, sol, ref))
    tr = s.trace()
    for col in ("rel_p", "rel_d", "merit", "sigma"):
        assert np.allclose(tr[:, hprlp.TRACE_COLS.index(col)], ref.trace_col(col), rtol=1e-9), col
    s.close()


@pytest.mark.parametrize("precision", [hprlp.FP64, hprlp.MIXED], ids=["fp64", "mixed"])
def test_bundles_full_solve(precision):
    from scipy.optimize import linprog
    import scipy.sparse as sp
    lp = transport()
    s = hprlp.Solver(lp, precision=precision)
    assert s.schedule(0)["bundle_items"] > 0
    sol = s.solve()
    assert sol.status == "OPTIMAL"
    A = sp.csr_matrix((lp.val, lp.colidx, lp.rowptr), shape=(lp.m, lp.n))
    h = linprog(lp.c, A_eq=A[:lp.m1], b_eq=lp.b[:lp.m1], A_ub=-A[lp.m1:], b_ub=-lp.b[lp.m1:],
                bounds=(0, None), method="highs")
    assert abs(sol.stats["pobj"] - h.fun) <= 1e-6 * (1 + abs(h.fun))
    from lp_truth import relative_kkt
    assert max(relative_kkt(lp, sol.x, sol.y, sol.z)) <= 1.5e-8
    s.close()


def test_forced_bundles_batched_with_compaction():
    parts = [dense(seed=610, m1=130, m2=130, n=300), dense(seed=611, m1=100, m2=170, n=290),
             lpgen.transport_lp(280, 66, seed=612)]
    lp = lpgen.pack_block_diagonal(parts, "bundles3")
    refs = [oracle.solve(p, max_iter=3000, check_every=100) for p in parts]
    s = hprlp.Solver(lp, batched=True, lambdas=[r.lam for r in refs], max_iter=3000,
                     check_every=100, bundle_rows=1)
    assert s.schedule(0)["bundle_items"] > 0 and s.schedule(1)["bundle_items"] > 0
    sol = s.solve()
    # instances stop at 1000, 1200 and 3000 iterations: the same stops, restarts and
    # statuses as the oracle, and the iterates at the 1e-10 bar norm-wise (over thousands of
    # iterations the rounding of small entries drifts past an entry-wise 1e-10)
    for i, ref in enumerate(refs):
        r0, r1 = lp.inst_row_off[i], lp.inst_row_off[i + 1]
        c0, c1 = lp.inst_col_off[i], lp.inst_col_off[i + 1]
        st = s.stats_instance(i)
        assert (st["iters"], st["restarts"], st["status"]) == (ref.iters, ref.restarts,
                                                               ref.status), i
        for name, a, b in (("x_bar", sol.x[c0:c1], ref.x), ("y_bar", sol.y[r0:r1], ref.y),
                           ("z_bar", sol.z[c0:c1], ref.z)):
            assert rel(a, b) <= 1e-10, (i, name, rel(a, b))
    print("iterations", [r.iters for r in refs], "compactions", sol.stats["n_compactions"])
    s.close()


def test_bundles_deterministic():
    lp = ot()
    a = hprlp.Solver(lp, max_iter=500, bundle_rows=1).solve()
    b = hprlp.Solver(lp, max_iter=500, bundle_rows=1).solve()
    for u, v in ((a.x, b.x), (a.y, b.y), (a.z, b.z)):
        assert np.array_equal(u.view(np.uint64), v.view(np.uint64))


@pytest.mark.parametrize("sched", ["default", "stress"])
def test_bundle_edges(sched):
    lp = edge_lp()
    ref = oracle.solve(lp, max_iter=100)
    extra = STRESS if sched == "stress" else {}
    s = hprlp.Solver(lp, max_iter=100, lambda_override=ref.lam, **extra)
    # 64 rows x 4 items (256 = 4 * 64), 2 rows x 5 items (300), 64 + 6 rows x 5 items (257)
    assert s.schedule(0)["bundle_items"] == 4 + 5 + 5 + 5, s.schedule(0)
    check(iterates(s, s.solve(), ref))
    s.close()


def test_short_shifted_rows_qap():
    """QAP LP (N = 20): its 16,000 rows of N + 1 = 21 nonzeros have columns r + N^3 k, so
    row r + 1's are row r's plus one: bundles of one work item each (21 <= 64 entries), whose
    epilogue runs in the item, one lane per row."""
    lp = lpgen.qap_lp(20, seed=1)
    ref = oracle.solve(lp, max_iter=100)
    s = hprlp.Solver(lp, max_iter=100, lambda_override=ref.lam)
    assert s.schedule(0)["bundle_items"] == expected_shifted_bundles(lp), s.schedule(0)
    check(iterates(s, s.solve(), ref))
    tr = s.trace()
    for col in ("rel_p", "rel_d", "merit"):
        assert np.allclose(tr[:, hprlp.TRACE_COLS.index(col)], ref.trace_col(col), rtol=1e-9), col
    s.close()
