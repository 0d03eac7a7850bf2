"""Pins of the oracle's T1 = 0 variant (Section 3.2, item 1: equality-only LPs, exact
y-step through A A^T, eq. sigma_T1=0), each against something other than the oracle:

  * A A^T = 4 I exactly (no scaling): T1 = lambda I - A A^T with lambda = 4 is then the zero
    operator, so the lambda-variant run with lambda = 4 must give the same iterates;
  * the first iteration from the origin: y_bar solves eq. AATy=R, checked with dense numpy;
  * the merit of that iteration equals d^T M d with M built densely from eq. def:M (T1 = 0);
  * full solves reach rel. KKT 1e-8 at the generator's certificate objective."""
import numpy as np
import pytest

import lpgen
from lp_truth import relative_kkt


def _orthogonal_rows_lp(m=20, extra=20, seed=5):
    """Rows with disjoint supports of 4 entries +-1: A A^T = 4 I exactly."""
    rng = np.random.default_rng(seed)
    n = 4 * m + extra
    rowptr = np.arange(m + 1, dtype=np.int64) * 4
    colidx = np.arange(4 * m, dtype=np.int32)
    val = rng.choice([-1.0, 1.0], size=4 * m)
    u = rng.uniform(1.0, 10.0, n)
    x0 = rng.uniform(0.0, 1.0, n) * u
    A = np.zeros((m, n))
    A[np.repeat(np.arange(m), 4), colidx] = val
    b = A @ x0
    c = rng.normal(size=n)
    return lpgen.LP("orth4", m, 0, n, rowptr, colidx, val, b, c, np.zeros(n), u), A


def _dense(lp):
    A = np.zeros((lp.m, lp.n))
    for i in range(lp.m):
        A[i, lp.colidx[lp.rowptr[i]:lp.rowptr[i + 1]]] = lp.val[lp.rowptr[i]:lp.rowptr[i + 1]]
    return A


def test_t1zero_equals_lambda_variant_when_AAT_is_lambda_I(oracle_mod):
    lp, A = _orthogonal_rows_lp()
    assert np.array_equal(A @ A.T, 4.0 * np.eye(lp.m))
    kw = dict(ruiz_iters=0, pock_chambolle=0, max_iter=3000, check_every=50)
    a = oracle_mod.solve(lp, t1_zero=1, **kw)
    b = oracle_mod.solve(lp, lambda_override=4.0, **kw)
    assert a.iters == b.iters and a.restarts == b.restarts and a.restarts > 2
    for u, v in ((a.x, b.x), (a.y, b.y), (a.x_cur, b.x_cur), (a.y_cur, b.y_cur)):
        assert np.linalg.norm(u - v) <= 1e-10 * max(np.linalg.norm(v), 1.0)
    # the sigma updates (eq. sigma_T1=0 against eq. sigma_T1!=0) agree too
    assert np.allclose(a.trace_col("sigma_new"), b.trace_col("sigma_new"), rtol=1e-10)


def _first_iteration(oracle_mod, lp):
    r = oracle_mod.solve(lp, t1_zero=1, max_iter=1)
    dr, dc = r.dr, r.dc
    At = dr[:, None] * _dense(lp) * dc[None, :]          # A~ = D_r A D_c
    bt = dr * lp.b / r.beta_b                            # b~
    xb = r.x / (r.beta_b * dc)                           # x_bar, scaled space
    yb = r.y / (r.beta_c * dr)                           # y_bar, scaled space
    return r, At, bt, xb, yb


@pytest.mark.parametrize("seed", [0, 1])
def test_t1zero_first_y_step_solves_AATy_R(oracle_mod, seed):
    lp = lpgen.bernoulli_lp(25, 0, 90, 0.12, seed=300 + seed)
    r, At, bt, xb, yb = _first_iteration(oracle_mod, lp)
    # from the origin with sigma = 1: A A^T y_bar = b - A(2 x_bar - 0)
    lhs = At @ (At.T @ yb)
    rhs = bt - At @ (2.0 * xb)
    assert np.linalg.norm(lhs - rhs) <= 1e-11 * max(np.linalg.norm(rhs), 1.0)


def test_t1zero_merit_is_the_M_norm(oracle_mod):
    lp = lpgen.bernoulli_lp(25, 0, 90, 0.12, seed=302)
    r, At, bt, xb, yb = _first_iteration(oracle_mod, lp)
    m, n = At.shape
    sigma = 1.0
    # M of eq. def:M with T1 = 0, on w = (y, x): [[sigma A A^T, A], [A^T, I / sigma]]
    M = np.block([[sigma * At @ At.T, At], [At.T, np.eye(n) / sigma]])
    # d = w^0 - w_hat^1 with w^0 = 0 and w_hat = 2 w_bar - w^0
    d = -2.0 * np.concatenate([yb, xb])
    merit = r.trace_col("merit")[0]
    assert np.isclose(merit, np.sqrt(d @ M @ d), rtol=1e-10)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_t1zero_full_solve_reaches_the_certificate(oracle_mod, seed):
    lp = lpgen.bernoulli_lp(30, 0, 120, 0.1, seed=310 + seed)
    r = oracle_mod.solve(lp, t1_zero=1)
    assert r.status == "OPTIMAL" and r.rel_kkt <= 1e-8
    assert abs(r.pobj - lp.cert.obj) <= 1e-7 * (1 + abs(lp.cert.obj))
    assert max(relative_kkt(lp, r.x, r.y, r.z)) <= 1.5e-8


def test_t1zero_rejects_inequality_rows(oracle_mod):
    lp = lpgen.bernoulli_lp(10, 5, 40, 0.2, seed=320)
    with pytest.raises(RuntimeError):
        oracle_mod.solve(lp, t1_zero=1)


@pytest.mark.parametrize("ns,nd", [(5, 7), (12, 15)])
def test_ot_generator_full_rank_and_feasible_coupling(ns, nd):
    lp = lpgen.ot_lp(ns, nd, seed=ns)
    A = _dense(lp)
    assert lp.m == ns + nd - 1 and lp.m2 == 0 and np.linalg.matrix_rank(A) == lp.m
    s, d = lp.b[:ns], np.concatenate([lp.b[ns:], [0.0]])
    d[-1] = s.sum() - d[:-1].sum()
    assert d[-1] > 0 and np.all(d > 0)
    x = (s[:, None] * d[None, :] / s.sum()).ravel()  # independent coupling
    assert np.allclose(A @ x, lp.b, rtol=1e-12)


def test_oracle_t1zero_on_ot_matches_highs(oracle_mod):
    from scipy.optimize import linprog
    import scipy.sparse as sp
    lp = lpgen.ot_lp(12, 15, seed=3)
    r = oracle_mod.solve(lp, t1_zero=1)
    assert r.status == "OPTIMAL"
    A = sp.csr_matrix((lp.val, lp.colidx, lp.rowptr), shape=(lp.m, lp.n))
    h = linprog(lp.c, A_eq=A, b_eq=lp.b, bounds=(0, None), method="highs")
    assert h.status == 0 and abs(r.pobj - h.fun) <= 1e-7 * (1 + abs(h.fun))
