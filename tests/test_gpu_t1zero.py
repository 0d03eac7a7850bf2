"""The T1 = 0 variant (Section 3.2, item 1) on the GPU, against the oracle running the same
variant: iterates after 100 and 700 iterations (restarts and sigma updates included) at the
1e-10 bar, the check trace, full solves, the rank check, and determinism.

The GPU applies the explicit inverse G of A~A~^T (one dense product per iteration) where
the oracle uses Cholesky solves; the scaled A~A~^T of these cases has condition number
5-160, so the two agree to ~1e-14 per step."""
import numpy as np
import pytest

import lpgen
import oracle
from paper_2408_12179_amd import hprlp

pytestmark = pytest.mark.gpu

STRESS = dict(tile_nnz=256, tile_rows=64, short_max=16, split_len=64, chunk_nnz=256)


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


def _case(name):
    if name == "bernoulli":
        return lpgen.bernoulli_lp(40, 0, 160, 0.08, seed=500)
    if name == "ot":
        return lpgen.ot_lp(20, 30, seed=501)
    if name == "ot_wide":
        return lpgen.ot_lp(60, 80, seed=502)
    return lpgen.zipf_lp(300, 0, 900, seed=503)


@pytest.mark.parametrize("iters", [100, 700])
@pytest.mark.parametrize("name", ["bernoulli", "ot", "ot_wide", "zipf"])
def test_t1zero_parity(name, iters):
    lp = _case(name)
    ref = oracle.solve(lp, t1_zero=1, max_iter=iters)
    s = hprlp.Solver(lp, t1_zero=1, max_iter=iters)
    sol = s.solve()
    assert sol.stats["iters"] == ref.iters and sol.stats["restarts"] == ref.restarts
    for k, a, b in (("x", sol.x, ref.x), ("y", sol.y, ref.y), ("z", sol.z, ref.z),
                    ("x_cur", s.iterate(hprlp.XCUR), ref.x_cur),
                    ("y_cur", s.iterate(hprlp.YCUR), ref.y_cur)):
        assert rel(a, b) <= 1e-10, (name, iters, k, rel(a, b))
    tr = s.trace()
    for col in ("sigma", "merit", "merit0"):
        got = tr[:, hprlp.TRACE_COLS.index(col)]
        assert np.allclose(got, ref.trace_col(col), rtol=1e-8), col
    s.close()


@pytest.mark.parametrize("opt", [dict(rho=1.6), STRESS], ids=["rho1.6", "stress"])
def test_t1zero_parity_options(opt):
    lp = _case("ot")
    ref = oracle.solve(lp, t1_zero=1, max_iter=400, **{k: v for k, v in opt.items() if k == "rho"})
    s = hprlp.Solver(lp, t1_zero=1, max_iter=400, **opt)
    sol = s.solve()
    assert sol.stats["iters"] == ref.iters and sol.stats["restarts"] == ref.restarts
    assert rel(sol.x, ref.x) <= 1e-10 and rel(sol.y, ref.y) <= 1e-10
    assert rel(s.iterate(hprlp.YCUR), ref.y_cur) <= 1e-10


def test_t1zero_full_solves():
    from scipy.optimize import linprog
    import scipy.sparse as sp
    lp = _case("bernoulli")
    sol = hprlp.Solver(lp, t1_zero=1).solve()
    assert sol.status == "OPTIMAL" and sol.stats["lambda"] == 0.0
    assert abs(sol.stats["pobj"] - lp.cert.obj) <= 1e-7 * (1 + abs(lp.cert.obj))
    lp = lpgen.ot_lp(30, 40, seed=504)
    ref = oracle.solve(lp, t1_zero=1)
    sol = hprlp.Solver(lp, t1_zero=1).solve()
    assert sol.status == "OPTIMAL" and sol.stats["iters"] == ref.iters
    A = sp.csr_matrix((lp.val, lp.colidx, lp.rowptr), shape=(lp.m, lp.n))
    h = linprog(lp.c, A_eq=A, b_eq=lp.b, bounds=(0, None), method="highs")
    assert abs(sol.stats["pobj"] - h.fun) <= 1e-6 * (1 + abs(h.fun))
    from lp_truth import relative_kkt
    assert max(relative_kkt(lp, sol.x, sol.y, sol.z)) <= 1.5e-8


def test_t1zero_rejects_rank_deficient_A():
    lp = lpgen.bernoulli_lp(20, 0, 80, 0.1, seed=505)
    # repeat row 0 as row 1: A A^T becomes singular
    r0 = slice(lp.rowptr[0], lp.rowptr[1])
    rows = [(lp.colidx[r0], lp.val[r0])] * 2 + [
        (lp.colidx[lp.rowptr[i]:lp.rowptr[i + 1]], lp.val[lp.rowptr[i]:lp.rowptr[i + 1]])
        for i in range(2, lp.m)]
    lp.rowptr = np.concatenate([[0], np.cumsum([len(c) for c, _ in rows])]).astype(np.int64)
    lp.colidx = np.concatenate([c for c, _ in rows]).astype(np.int32)
    lp.val = np.concatenate([v for _, v in rows])
    lp.b[1] = lp.b[0]
    with pytest.raises(hprlp.HPRLPError) as e:
        hprlp.Solver(lp, t1_zero=1)
    assert e.value.code == hprlp.EINVAL and "full row rank" in str(e.value)


def test_t1zero_deterministic():
    lp = _case("ot_wide")
    a = hprlp.Solver(lp, t1_zero=1, max_iter=500).solve()
    b = hprlp.Solver(lp, t1_zero=1, max_iter=500).solve()
    for u, v in ((a.x, b.x), (a.y, b.y), (a.z, b.z)):
        assert np.array_equal(u.view(np.uint64), v.view(np.uint64))


def test_t1zero_parity_ot_512():
    """m = 1023: 16 panels of the blocked sweep, the last one padded; the residual pass
    runs the demand rows (511 of 512 nonzeros, columns shifted by one) as row bundles."""
    lp = lpgen.ot_lp(512, 512, seed=506)
    ref = oracle.solve(lp, t1_zero=1, max_iter=100)
    s = hprlp.Solver(lp, t1_zero=1, max_iter=100)
    assert s.schedule(0)["bundle_items"] > 0
    sol = s.solve()
    assert sol.stats["iters"] == ref.iters == 100
    for k, a, b in (("x", sol.x, ref.x), ("y", sol.y, ref.y), ("z", sol.z, ref.z),
                    ("y_cur", s.iterate(hprlp.YCUR), ref.y_cur)):
        assert rel(a, b) <= 1e-10, (k, rel(a, b))
    s.close()
