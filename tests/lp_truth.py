"""Ground truth that does not come from the oracle: exhaustive vertex enumeration, the
generator's KKT certificate, and dense-matrix forms of the paper's definitions.  Test
infrastructure only."""
from __future__ import annotations

import itertools

import numpy as np


def vertex_enumeration(lp):
    """Exact optimum of a small LP with every column boxed, by enumerating all vertices:
    each vertex is the solution of n linearly independent active constraints taken from the
    equality rows (always active), the inequality rows and the bounds."""
    A = lp.dense()
    m1, n = lp.m1, lp.n
    assert np.all(np.isfinite(lp.l)) and np.all(np.isfinite(lp.u))
    rows, rhs = [], []
    for i in range(m1, lp.m):
        rows.append(A[i]); rhs.append(lp.b[i])
    for j in range(n):
        e = np.zeros(n); e[j] = 1.0
        rows.append(e); rhs.append(lp.l[j])
        rows.append(e.copy()); rhs.append(lp.u[j])
    rows, rhs = np.array(rows), np.array(rhs)
    best, best_x = np.inf, None
    k = n - m1
    for S in itertools.combinations(range(len(rows)), k):
        M = np.vstack([A[:m1], rows[list(S)]])
        r = np.concatenate([lp.b[:m1], rhs[list(S)]])
        if abs(np.linalg.det(M)) < 1e-10:
            continue
        x = np.linalg.solve(M, r)
        tol = 1e-9 * (1 + np.abs(x).max())
        if np.any(x < lp.l - tol) or np.any(x > lp.u + tol):
            continue
        Ax = A @ x
        if np.any(np.abs(Ax[:m1] - lp.b[:m1]) > 1e-8 * (1 + np.abs(lp.b[:m1]).max(initial=0))):
            continue
        if np.any(Ax[m1:] < lp.b[m1:] - tol * (1 + np.abs(lp.b).max())):
            continue
        obj = float(lp.c @ x)
        if obj < best:
            best, best_x = obj, x
    return best, best_x


def support_box(z, l, u):
    """delta*_C(-z) = sum_j max(-z_j,0) u_j - max(z_j,0) l_j with 0 * inf = 0."""
    zp, zm = np.maximum(z, 0), np.maximum(-z, 0)
    a = zm * np.where(zm == 0, 0.0, u)
    b = zp * np.where(zp == 0, 0.0, l)
    return float(np.sum(a) - np.sum(b))


def relative_kkt(lp, x, y, z):
    """(rel_p, rel_d, rel_gap) of a primal-dual point on the original data, written from the
    termination inequalities of Section 4.1 with dense numpy algebra."""
    A = lp.dense() if lp.n * lp.m <= 4e6 else None
    if A is not None:
        Ax, Aty = A @ x, A.T @ y
    else:
        row_of = np.repeat(np.arange(lp.m), np.diff(lp.rowptr))
        Ax = np.bincount(row_of, weights=lp.val * x[lp.colidx], minlength=lp.m)
        Aty = np.bincount(lp.colidx, weights=lp.val * y[row_of], minlength=lp.n)
    r = lp.b - Ax
    ineq = ~lp.eq_mask()
    r[ineq] = np.maximum(r[ineq], 0)
    rel_p = np.linalg.norm(r) / (1 + np.linalg.norm(lp.b))
    rel_d = np.linalg.norm(lp.c - Aty - z) / (1 + np.linalg.norm(lp.c))
    dobj = float(lp.b @ y) - support_box(z, lp.l, lp.u)
    pobj = float(lp.c @ x)
    gap = abs(dobj - pobj) / (1 + abs(dobj) + abs(pobj))
    return rel_p, rel_d, gap


def dense_M(At, lam, sigma):
    """The operator M of eq. def:M as a dense matrix on w = (y, z, x), with
    T1 = lam I - A A^T (Section 3.2, second choice)."""
    m, n = At.shape
    T1 = lam * np.eye(m) - At @ At.T
    M = np.zeros((m + 2 * n, m + 2 * n))
    M[:m, :m] = sigma * (At @ At.T) + sigma * T1
    M[:m, m + n:] = At
    M[m + n:, :m] = At.T
    M[m + n:, m + n:] = np.eye(n) / sigma
    return M
