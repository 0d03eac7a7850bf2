"""The QAP LP workload (Section 4.4: the Adams-Johnson form the paper writes out) and the
oracle on it.

Generator pins: the closed-form sizes, and for random permutations pi the point
x_ij = [pi(i) = j], s_ijkl = x_ij x_kl solves every row exactly and costs
sum_ik a_ik b_pi(i)pi(k), the QAP objective of pi (so the LP is a relaxation of the QAP).
Oracle pins: on N = 3 and 4 the oracle reaches rel. KKT 1e-8, its objective matches the LP
optimum of HiGHS (scipy), and it is at most the QAP optimum found by brute force."""
import itertools

import numpy as np
import pytest
import scipy.sparse as sp

import lpgen
from lp_truth import relative_kkt


def _csr(lp):
    return sp.csr_matrix((lp.val, lp.colidx, lp.rowptr), shape=(lp.m, lp.n))


@pytest.mark.parametrize("N", [2, 3, 5, 8])
def test_qap_sizes(N):
    lp = lpgen.qap_lp(N, seed=1)
    assert lp.m1 == 2 * N ** 3 + N * N * (N * N - 1) // 2 + 2 * N and lp.m2 == 0
    assert lp.n == N ** 4 + N ** 2
    assert lp.nnz == 2 * N ** 3 * (N + 1) + N * N * (N * N - 1) + 2 * N * N
    for i in range(lp.m):  # strictly increasing columns: no repeats in a row
        assert np.all(np.diff(lp.colidx[lp.rowptr[i]:lp.rowptr[i + 1]]) > 0)
    assert np.all(lp.val == lp.val.astype(np.float32)) and np.all(lp.c == lp.c.astype(np.float32))


@pytest.mark.parametrize("N", [3, 5, 7])
def test_qap_permutations_are_feasible_with_the_qap_cost(N):
    lp = lpgen.qap_lp(N, seed=2)
    a, b = lp.meta["flow"], lp.meta["dist"]
    A = _csr(lp)
    rng = np.random.default_rng(3)
    for _ in range(4):
        pi = rng.permutation(N)
        X = np.zeros((N, N))
        X[np.arange(N), pi] = 1.0
        S = np.einsum("ij,kl->ijkl", X, X)
        w = np.concatenate([S.ravel(), X.ravel()])
        assert np.array_equal(A @ w, lp.b)  # integer data: exact
        assert np.all(w >= lp.l) and np.all(w <= lp.u)
        qap_cost = sum(a[i, k] * b[pi[i], pi[k]] for i in range(N) for k in range(N))
        assert lp.c @ w == qap_cost


@pytest.mark.parametrize("N", [3, 4])
def test_oracle_on_qap_matches_highs_and_bounds_the_qap(N):
    import oracle
    from scipy.optimize import linprog
    lp = lpgen.qap_lp(N, seed=4)
    r = oracle.solve(lp, max_iter=2_000_000)
    assert r.status == "OPTIMAL" and r.rel_kkt <= 1e-8
    rp, rd, gap = relative_kkt(lp, r.x, r.y, r.z)
    assert max(rp, rd, gap) <= 1.5e-8
    h = linprog(lp.c, A_eq=_csr(lp), b_eq=lp.b,
                bounds=list(zip(lp.l, np.where(np.isinf(lp.u), None, lp.u))), method="highs")
    assert h.status == 0
    assert abs(r.pobj - h.fun) <= 1e-6 * (1 + abs(h.fun)), (r.pobj, h.fun)
    a, b = lp.meta["flow"], lp.meta["dist"]
    best = min(sum(a[i, k] * b[p[i], p[k]] for i in range(N) for k in range(N))
               for p in itertools.permutations(range(N)))
    assert r.pobj <= best + 1e-6 * (1 + best), (r.pobj, best)
