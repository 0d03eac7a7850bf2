"""Pins of the CPU oracle against things other than itself (CPU only).

Each test ties one part of the oracle to an independent truth:
  * exhaustive vertex enumeration on tiny boxed LPs                (final answer)
  * the generator's constructed KKT certificate                    (final answer)
  * scipy's HiGHS                                                  (final answer)
  * numpy's symmetric eigensolver                                  (power method)
  * closed forms of Ruiz / Pock-Chambolle scaling                  (preconditioning)
  * a textbook Chambolle-Pock PDHG step (Halpern off, rho = 1)      (one iteration's map)
  * the dense operator M of eq. def:M                              (restart merit)
  * eq. sigma with a dense T1                                      (SigmaUpdate)
  * Proposition 2.3 and Theorem 2.4 bounds along the iteration     (whole Halpern loop)
"""
import numpy as np
import pytest

import lpgen
from lp_truth import dense_M, relative_kkt, support_box, vertex_enumeration


# ----------------------------------------------------------------------------- generator

@pytest.mark.parametrize("name,scale", [("tiny", 1), ("zipf1m", 0.004), ("batch256", 0.01)])
def test_generator_certificate_is_kkt(name, scale):
    lp = lpgen.make(name, scale)
    x, y, z = lp.cert.x, lp.cert.y, lp.cert.z
    A = lp.dense()
    assert np.all(x >= lp.l) and np.all(x <= lp.u)
    r = A @ x - lp.b
    eq = lp.eq_mask()
    assert np.allclose(r[eq], 0, atol=1e-10)
    assert np.all(r[~eq] >= -1e-10)
    assert np.all(y[~eq] >= 0)
    assert np.allclose(y[~eq] * r[~eq], 0, atol=1e-10)  # complementary slackness
    assert np.allclose(A.T @ y + z, lp.c, atol=1e-10)
    assert np.all(z[x > lp.l] <= 0) and np.all(z[x < lp.u] >= 0)
    # strong duality: <c, x0> = <b, y0> - delta*_C(-z0)
    dobj = lp.b @ y - support_box(z, lp.l, lp.u)
    assert abs(dobj - lp.cert.obj) <= 1e-9 * (1 + abs(lp.cert.obj))
    assert max(relative_kkt(lp, x, y, z)) < 1e-12


def test_generator_fp32_exact_and_shapes():
    lp = lpgen.make("zipf1m", 0.004)
    assert np.all(lp.val.astype(np.float32).astype(np.float64) == lp.val)
    lens = np.diff(lp.rowptr)
    assert lens.min() >= 5 and lens.max() <= 40
    for i in range(0, lp.m, 97):  # no repeated column inside a row
        cols = lp.colidx[lp.rowptr[i]:lp.rowptr[i + 1]]
        assert len(np.unique(cols)) == len(cols)
    free = ~np.isfinite(lp.l)
    assert 0.25 < free.mean() < 0.35
    t = lpgen.make("transport10m", 0.01)
    assert t.b[:t.m1].sum() >= t.b[t.m1:].sum()
    assert np.all(np.diff(t.rowptr)[:t.m1] == 50) and np.all(np.diff(t.rowptr)[t.m1:] == 20)


# ----------------------------------------------------------------------------- final answers

@pytest.mark.parametrize("seed", range(6))
def test_oracle_matches_vertex_enumeration(oracle_mod, seed):
    m1 = seed % 3
    lp = lpgen.tiny_boxed_lp(m1, 2 + seed % 2, 4 + seed % 4, seed=100 + seed)
    best, _ = vertex_enumeration(lp)
    assert np.isfinite(best)
    r = oracle_mod.solve(lp, tol=1e-10, max_iter=400000)
    assert r.status == "OPTIMAL"
    assert abs(r.pobj - best) <= 1e-8 * (1 + abs(best)), (r.pobj, best)


def test_oracle_tiny_matches_certificate_and_highs(oracle_mod):
    from scipy.optimize import linprog
    lp = lpgen.make("tiny")
    r = oracle_mod.solve(lp)
    assert r.status == "OPTIMAL" and r.rel_kkt <= 1e-8
    assert abs(r.pobj - lp.cert.obj) <= 1e-7 * (1 + abs(lp.cert.obj))
    A = lp.dense()
    h = linprog(lp.c, A_ub=-A[lp.m1:], b_ub=-lp.b[lp.m1:], A_eq=A[:lp.m1], b_eq=lp.b[:lp.m1],
                bounds=list(zip(lp.l, np.where(np.isinf(lp.u), None, lp.u))), method="highs")
    assert h.status == 0
    assert abs(r.pobj - h.fun) <= 1e-7 * (1 + abs(h.fun))
    # the oracle's own KKT numbers agree with an independent dense evaluation
    rp, rd, gap = relative_kkt(lp, r.x, r.y, r.z)
    assert np.isclose(rp, r.rel_p, rtol=1e-6, atol=1e-14)
    assert np.isclose(rd, r.rel_d, rtol=1e-6, atol=1e-14)
    assert np.isclose(gap, r.rel_gap, rtol=1e-6, atol=1e-14)


@pytest.mark.parametrize("name,scale", [("zipf1m", 0.0005), ("batch256", 0.004)])
def test_oracle_downscaled_matches_certificate(oracle_mod, name, scale):
    lp = lpgen.make(name, scale)
    r = oracle_mod.solve(lp, max_iter=300000)
    assert r.status == "OPTIMAL"
    assert abs(r.pobj - lp.cert.obj) <= 1e-7 * (1 + abs(lp.cert.obj))


def test_oracle_transport_matches_highs(oracle_mod):
    from scipy.optimize import linprog
    from scipy.sparse import csr_matrix
    lp = lpgen.make("transport10m", 0.006)  # 12 x 30
    A = csr_matrix((lp.val, lp.colidx, lp.rowptr), shape=(lp.m, lp.n))
    h = linprog(lp.c, A_ub=-A[lp.m1:], b_ub=-lp.b[lp.m1:], A_eq=A[:lp.m1], b_eq=lp.b[:lp.m1],
                bounds=(0, None), method="highs")
    r = oracle_mod.solve(lp, max_iter=300000)
    assert r.status == "OPTIMAL"
    assert abs(r.pobj - h.fun) <= 1e-7 * (1 + abs(h.fun))


# ----------------------------------------------------------------------------- power method

@pytest.mark.parametrize("seed", range(3))
def test_power_method_matches_eigvalsh(oracle_mod, seed):
    lp = lpgen.bernoulli_lp(20, 15, 40, 0.2, seed=seed)
    S = oracle_mod.scale(lp)
    At = lpgen.LP("s", lp.m1, lp.m2, lp.n, lp.rowptr, lp.colidx, S.val, lp.b, lp.c, lp.l,
                  lp.u).dense()
    ev = np.linalg.eigvalsh(At @ At.T)
    lam, it = oracle_mod.power(lp.m, lp.n, lp.rowptr, lp.colidx, S.val, max_iter=200000,
                               tol=1e-15)
    assert abs(lam - ev[-1]) <= 1e-9 * ev[-1]
    # Rayleigh quotients never exceed lambda_max; Pock-Chambolle (alpha=1) bounds ||A~|| by 1
    assert lam <= ev[-1] * (1 + 1e-14)
    assert ev[-1] <= 1 + 1e-12


# ----------------------------------------------------------------------------- scaling

def _lp_from_dense(D, m1=None):
    m, n = D.shape
    mask = D != 0
    rowptr = np.concatenate([[0], np.cumsum(mask.sum(1))]).astype(np.int64)
    col = np.concatenate([np.nonzero(mask[i])[0] for i in range(m)]).astype(np.int32)
    return lpgen.LP("d", m if m1 is None else m1, 0 if m1 is None else m - m1, n, rowptr,
                    col, D[mask], np.ones(m), np.ones(n), np.zeros(n), np.full(n, np.inf))


def test_scaling_diagonal_closed_form(oracle_mod):
    a = np.array([4.0, -0.25, 9.0, 1e-6, -3e5])
    S = oracle_mod.scale(_lp_from_dense(np.diag(a)))
    assert np.array_equal(S.val, np.sign(a))
    assert np.allclose(S.dr * S.dc * np.abs(a), 1.0, rtol=1e-15)


def test_scaling_transport_closed_form(oracle_mod):
    # every |a_ij| equal: Ruiz maps all entries to +-1, then Pock-Chambolle with alpha=1
    # divides each entry by sqrt(row length * column length)
    lp = lpgen.transport_lp(3, 7, seed=5)
    lp.val = lp.val * 6.25
    S = oracle_mod.scale(lp)
    lens = np.diff(lp.rowptr)
    row_of = np.repeat(np.arange(lp.m), lens)
    collen = np.bincount(lp.colidx, minlength=lp.n)
    want = 1.0 / np.sqrt(lens[row_of] * collen[lp.colidx])
    assert np.allclose(S.val, want, rtol=1e-14)


def test_scaling_ruiz_equilibrates_and_reconstructs(oracle_mod):
    lp = lpgen.bernoulli_lp(30, 30, 80, 0.1, seed=3)
    lp.val = lp.val * np.exp(np.random.default_rng(0).uniform(-6, 6, lp.nnz))
    S = oracle_mod.scale(lp, pock_chambolle=0)
    D = lp.dense()
    Ds = np.diag(S.dr) @ D @ np.diag(S.dc)
    row_of = np.repeat(np.arange(lp.m), np.diff(lp.rowptr))
    assert np.allclose(Ds[row_of, lp.colidx], S.val, rtol=1e-13)
    rmax = np.abs(Ds).max(axis=1)
    cmax = np.abs(Ds).max(axis=0)
    assert np.all(np.abs(rmax[rmax > 0] - 1) < 1e-2)
    assert np.all(np.abs(cmax[cmax > 0] - 1) < 1e-2)
    # b and c normalisation: scaled data divided by (norm + 1)
    assert np.isclose(np.linalg.norm(S.b), np.linalg.norm(S.dr * lp.b) / S.beta_b)
    assert np.isclose(S.beta_b, np.linalg.norm(S.dr * lp.b) + 1)
    assert np.isclose(S.beta_c, np.linalg.norm(S.dc * lp.c) + 1)


# ----------------------------------------------------------------------------- one iteration

def _scaled_dense(oracle_mod, lp):
    S = oracle_mod.scale(lp)
    At = lpgen.LP("s", lp.m1, lp.m2, lp.n, lp.rowptr, lp.colidx, S.val, lp.b, lp.c, lp.l,
                  lp.u).dense()
    return S, At


def test_one_step_is_textbook_pdhg(oracle_mod):
    """With the Halpern step off and rho = 1 (no reflection), an iteration of eqs. update-x
    and update-y-2 is a Chambolle-Pock primal-dual step with primal step tau = sigma and dual
    step s = 1 / (lambda sigma) on min_x max_{y in D} <c,x> - <y, A x - b>."""
    lp = lpgen.make("tiny")
    S, At = _scaled_dense(oracle_mod, lp)
    lam = float(np.linalg.eigvalsh(At @ At.T)[-1])
    sigma = 0.7
    K = 37
    r = oracle_mod.solve(lp, use_halpern=0, rho=1.0, use_restart=0, sigma_update=0,
                         sigma0=sigma, lambda_override=lam, max_iter=K)
    tau, s = sigma, 1.0 / (lam * sigma)
    x, y = np.zeros(lp.n), np.zeros(lp.m)
    for _ in range(K):
        x_new = np.clip(x - tau * (S.c - At.T @ y), S.l, S.u)
        y_new = y + s * (S.b - At @ (2 * x_new - x))
        y_new[lp.m1:] = np.maximum(y_new[lp.m1:], 0)
        x, y = x_new, y_new
    assert np.allclose(r.x_cur / (S.beta_b * S.dc), x, rtol=1e-11, atol=1e-13)
    assert np.allclose(r.y_cur / (S.beta_c * S.dr), y, rtol=1e-11, atol=1e-13)


def test_merit_equals_dense_M_norm(oracle_mod):
    """R~ = ||w - w_hat||_M with M written out densely from eq. def:M."""
    lp = lpgen.make("tiny")
    S, At = _scaled_dense(oracle_mod, lp)
    lam = float(np.linalg.eigvalsh(At @ At.T)[-1])
    K = 23
    kw = dict(use_restart=0, sigma_update=0, sigma0=1.3, lambda_override=lam)
    a = oracle_mod.solve(lp, max_iter=K, **kw)                      # w^K
    b = oracle_mod.solve(lp, max_iter=K + 1, trace_every_iter=1, iter_cap=K + 1, **kw)
    w = np.concatenate([a.y_cur / (S.beta_c * S.dr), np.zeros(lp.n), a.x_cur / (S.beta_b * S.dc)])
    wbar = np.concatenate([b.y / (S.beta_c * S.dr), b.z * S.dc / S.beta_c, b.x / (S.beta_b * S.dc)])
    d = w - (2 * wbar - w)
    M = dense_M(At, lam, 1.3)
    assert np.isclose(np.sqrt(d @ M @ d), b.iter_trace[K, 0], rtol=1e-10)


def test_sigma_update_matches_eq_sigma(oracle_mod):
    """The first restart (k = 150) sets sigma = Delta_x / Delta_y; with a dense T1 this must
    equal sqrt(||dx||^2 / (||dy||^2_T1 + ||A^T dy||^2)) of eqs. sigma, Dx&Dy."""
    lp = lpgen.make("tiny")
    S, At = _scaled_dense(oracle_mod, lp)
    a = oracle_mod.solve(lp, max_iter=150)
    b = oracle_mod.solve(lp, max_iter=151)
    row = b.trace[0]
    assert row[0] == 150 and row[16] == 1.0  # first check restarts (criterion 3, t = k)
    lam = b.lam
    xb = a.x / (S.beta_b * S.dc)
    yb = a.y / (S.beta_c * S.dr)
    dx, dy = xb - 0.0, yb - 0.0  # anchors of the first outer loop are the origin
    T1 = lam * np.eye(lp.m) - At @ At.T
    sig = np.sqrt(dx @ dx / (dy @ T1 @ dy + np.sum((At.T @ dy) ** 2)))
    assert np.isclose(row[17], sig, rtol=1e-9)


# ----------------------------------------------------------------------------- invariants

def test_halpern_bounds_prop23_thm24(oracle_mod):
    """Fixed sigma, no restart: along the whole run
       ||w^k - w_hat^{k+1}||_M <= 2 ||w^0 - w*||_M / (k+1)                (Prop. 2.3)
       ||R(w_bar^{k+1})|| <= (sigma(||A||+||sqrt T1||)+1)/sqrt(sigma) R0/(k+1)  (Thm. 2.4)
    with w* the scaled certificate and lambda = lambda_1(A A^T) exactly; also x_bar in C and
    y_bar in D at every iteration (Section 4.1)."""
    lp = lpgen.make("tiny")
    S, At = _scaled_dense(oracle_mod, lp)
    ev = np.linalg.eigvalsh(At @ At.T)
    lam = float(ev[-1])
    sigma = 0.9
    K = 3000
    r = oracle_mod.solve(lp, max_iter=K, use_restart=0, sigma_update=0, sigma0=sigma,
                         lambda_override=lam, trace_every_iter=1, iter_cap=K)
    ys = lp.cert.y / (S.beta_c * S.dr)
    xs = lp.cert.x / (S.beta_b * S.dc)
    wstar = np.concatenate([ys, np.zeros(lp.n), xs])
    M = dense_M(At, lam, sigma)
    R0 = np.sqrt(wstar @ M @ wstar)
    k = np.arange(K)
    merit, kkt = r.iter_trace[:, 0], r.iter_trace[:, 1]
    assert np.all(merit <= 2 * R0 / (k + 1) * (1 + 1e-9))
    const = (sigma * (np.sqrt(lam) + np.sqrt(max(lam - ev[0], 0))) + 1) / np.sqrt(sigma)
    assert np.all(kkt <= const * R0 / (k + 1) * (1 + 1e-9))
    assert np.all(r.iter_trace[:, 2] <= 0) and np.all(r.iter_trace[:, 3] <= 0)


# ----------------------------------------------------------------------------- control flow

def test_first_restart_at_first_check_and_statuses(oracle_mod):
    lp = lpgen.make("tiny")
    r = oracle_mod.solve(lp, max_iter=1)
    assert r.status == "ITER_LIMIT" and r.iters == 1
    r = oracle_mod.solve(lp, max_iter=1000)
    assert r.status == "ITER_LIMIT"
    assert r.trace[0, 0] == 150 and r.trace[0, 16] == 1
    # every check before termination evaluated the criteria on the recorded merits
    for row in r.trace[:-1]:
        k, t = row[0], row[1]
        fired = (row[4] <= 0.2 * row[5]) or (row[4] <= 0.6 * row[5] and row[4] > row[6]) \
            or t >= 0.2 * k
        assert bool(row[16]) == fired


def test_infeasible_lp_hits_iteration_limit(oracle_mod):
    # x1 + x2 = 3 with 0 <= x <= 1: infeasible; the method has no infeasibility detection
    D = np.array([[1.0, 1.0]])
    lp = _lp_from_dense(D, m1=1)
    lp.b = np.array([3.0]); lp.c = np.array([1.0, 2.0]); lp.u = np.ones(2)
    r = oracle_mod.solve(lp, max_iter=3000)
    assert r.status == "ITER_LIMIT" and r.rel_p > 1e-3
