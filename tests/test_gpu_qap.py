"""The HIP path on the QAP LP workload (Section 4.4 form; all rows equalities, columns of
3 nonzeros next to columns of 2N + 2): iterate parity with the oracle, across restarts,
and full solves against the oracle's and HiGHS's optimal values."""
import numpy as np
import pytest

import lpgen
import oracle
from paper_2408_12179_amd import hprlp

pytestmark = pytest.mark.gpu


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


@pytest.mark.parametrize("N,iters", [(6, 700), (10, 100), (13, 100)])
def test_qap_iterate_parity(N, iters):
    lp = lpgen.qap_lp(N, seed=7)
    ref = oracle.solve(lp, max_iter=iters)
    s = hprlp.Solver(lp, max_iter=iters, lambda_override=ref.lam)
    sol = s.solve()
    assert sol.stats["iters"] == ref.iters and sol.stats["restarts"] == ref.restarts
    for k, a, b in (("x", sol.x, ref.x), ("y", sol.y, ref.y), ("z", sol.z, ref.z),
                    ("x_cur", s.iterate(hprlp.XCUR), ref.x_cur),
                    ("y_cur", s.iterate(hprlp.YCUR), ref.y_cur)):
        assert rel(a, b) <= 1e-10, (N, k, rel(a, b))
    s.close()


@pytest.mark.parametrize("prec", [hprlp.FP64, hprlp.MIXED])
def test_qap_full_solve(prec):
    from scipy.optimize import linprog
    import scipy.sparse as sp
    lp = lpgen.qap_lp(5, seed=8)
    ref = oracle.solve(lp, max_iter=2_000_000)
    sol = hprlp.Solver(lp, precision=prec).solve()
    st = sol.stats
    assert sol.status == "OPTIMAL" and max(st["rel_p"], st["rel_d"], st["rel_gap"]) <= 1e-8
    assert abs(st["pobj"] - ref.pobj) <= 1e-7 * (1 + abs(ref.pobj))
    A = sp.csr_matrix((lp.val, lp.colidx, lp.rowptr), shape=(lp.m, lp.n))
    h = linprog(lp.c, A_eq=A, b_eq=lp.b,
                bounds=list(zip(lp.l, np.where(np.isinf(lp.u), None, lp.u))), method="highs")
    assert h.status == 0 and abs(st["pobj"] - h.fun) <= 1e-6 * (1 + abs(h.fun))
    from lp_truth import relative_kkt
    assert max(relative_kkt(lp, sol.x, sol.y, sol.z)) <= 1.5e-8
