"""Pins of the oracle's restart and sigma machinery and of its bound handling (CPU only).

  * SigmaUpdate's safeguard (Algorithm 3 with eqs. Dx_Dy and primal_dual_infeasibility,
    Section 3.2): inputs that drive the first restart into the "otherwise sigma := 1" branch
    through each of its conditions (Delta_x <= 1e-16, Delta_y <= 1e-16 with err_p = 0, and
    err_d / err_p above 1e8 or below 1e-8), with Delta_x, Delta_y, err_p and err_d recomputed
    in numpy from the returned w_bar and the scaled data, and sigma0 != 1 so that a reset to
    sigma0 or no reset would both fail.
  * The restart bookkeeping of Section 3.1 (readings A1, A2): the merit R~_{r,0} and the
    previous-check merit each check compares with, rebuilt from the merit of every
    iteration, and the restart decisions re-taken from criteria 1-3; runs that restart by
    criterion 1 alone and by criterion 2 alone are included.
  * The Halpern weight of Algorithm 2 at t = 0: one Halpern iteration from the origin is half
    of one plain Peaceman-Rachford iteration.
  * Every kind of column bound (eq. update-x, delta*_C of Section 4.1): the oracle's optimum on
    LPs with boxed, fixed (l = u), lower-only, upper-only and free columns equals the
    generator's certificate and scipy's HiGHS.
  * The OpenMP build of the oracle (used only to time it on all cores) gives the plain build's
    results bit for bit.
"""
import numpy as np
import pytest

import lpgen

TR = ["k", "t", "r", "sigma", "merit", "merit0", "merit_prev", "rel_p", "rel_d", "rel_gap",
      "pobj", "dobj", "dx", "dy", "err_p", "err_d", "restart", "sigma_new"]
C = {k: i for i, k in enumerate(TR)}


def sigma_cases():
    """(name, lp, sigma0) whose first restart (k = 150) takes the sigma := 1 branch."""
    fixed0 = lpgen.bernoulli_lp(6, 6, 20, 0.3, seed=100)
    fixed0.l = np.zeros(fixed0.n)  # every column fixed at 0 and b != 0: infeasible, x_bar = 0
    fixed0.u = np.zeros(fixed0.n)
    slack = lpgen.bernoulli_lp(0, 12, 20, 0.3, seed=100)
    slack.b = np.full(slack.m, -1e3)  # inequality rows never violated: y stays 0, err_p = 0
    slack.u = np.full(slack.n, 1.0)
    # small costs: x crawls towards its bounds, so the dual residual stays near 1e-5 through
    # both restarts instead of reaching rounding level (where either side may stop as optimal)
    slack.c = slack.c * 1e-5
    base = lpgen.bernoulli_lp(6, 6, 20, 0.3, seed=100)
    return [("dx_zero", fixed0, 3.0), ("dy_zero_errp_zero", slack, 3.0),
            ("ratio_above_1e8", base, 1e-9), ("ratio_below_1e-8", base, 1e9)]


def _restart_quantities(oracle_mod, lp, sigma0):
    """Delta_x, Delta_y, err_p, err_d at k = 150 recomputed from w_bar (Section 3.2, eq.
    sigma_T1!=0 and the residuals of the safeguard), on the scaled problem of Section 4.1."""
    S = oracle_mod.scale(lp)
    At = lpgen.LP("s", lp.m1, lp.m2, lp.n, lp.rowptr, lp.colidx, S.val, lp.b, lp.c, lp.l,
                  lp.u).dense()
    a = oracle_mod.solve(lp, max_iter=150, sigma0=sigma0, tol=1e-30)
    xb = a.x / (S.beta_b * S.dc)
    yb = a.y / (S.beta_c * S.dr)
    zb = a.z * S.dc / S.beta_c
    dx = np.linalg.norm(xb)                    # the anchors of the first loop are the origin
    dy = np.sqrt(a.lam) * np.linalg.norm(yb)
    r = S.b - At @ xb
    r[lp.m1:] = np.maximum(r[lp.m1:], 0.0)     # Pi_D: inequality rows count where violated
    err_p = np.linalg.norm(r) / (1 + np.linalg.norm(S.b))
    err_d = np.linalg.norm(S.c - At.T @ yb - zb) / (1 + np.linalg.norm(S.c))
    return dx, dy, err_p, err_d


@pytest.mark.parametrize("case", range(4))
def test_sigma_reset_branch(oracle_mod, case):
    name, lp, s0 = sigma_cases()[case]
    r = oracle_mod.solve(lp, max_iter=301, sigma0=s0, tol=1e-30)
    row = r.trace[0]
    assert row[C["k"]] == 150 and row[C["restart"]] == 1.0 and row[C["sigma"]] == s0
    dx, dy, ep, ed = _restart_quantities(oracle_mod, lp, s0)
    for got, want in ((row[C["dx"]], dx), (row[C["dy"]], dy), (row[C["err_p"]], ep),
                      (row[C["err_d"]], ed)):
        assert abs(got - want) <= 1e-9 * max(abs(want), 1e-300) + 1e-300, (name, got, want)
    ok_dx = 1e-16 < dx < 1e12
    ok_dy = 1e-16 < dy < 1e12
    ratio_ok = ep > 0 and 1e-8 < ed / ep < 1e8
    if name == "dx_zero":
        assert dx == 0.0 and ok_dy and ratio_ok
    elif name == "dy_zero_errp_zero":
        assert dy == 0.0 and ep == 0.0 and ok_dx
    else:
        assert ok_dx and ok_dy and not ratio_ok
        assert (ed / ep > 1e8) == (name == "ratio_above_1e8")
    # the safeguard fails: sigma := 1, not sigma0 and not Delta_x / Delta_y
    assert row[C["sigma_new"]] == 1.0
    assert r.trace[1, C["sigma"]] == 1.0


def test_sigma_in_band_control(oracle_mod):
    """Same LP, sigma0 = 1: every condition holds and sigma = Delta_x / Delta_y != 1."""
    lp = sigma_cases()[2][1]
    r = oracle_mod.solve(lp, max_iter=151, tol=1e-30)
    dx, dy, ep, ed = _restart_quantities(oracle_mod, lp, 1.0)
    assert 1e-16 < dx < 1e12 and 1e-16 < dy < 1e12 and 1e-8 < ed / ep < 1e8
    assert np.isclose(r.trace[0, C["sigma_new"]], dx / dy, rtol=1e-9)
    assert abs(r.trace[0, C["sigma_new"]] - 1.0) > 1e-3


def _criteria_pin(oracle_mod, lp, kmax, ce=150):
    """Rebuild merit0 and merit_prev of every check from the per-iteration merits and re-take
    each restart decision; returns which criteria fired alone."""
    r = oracle_mod.solve(lp, max_iter=kmax, iter_cap=kmax, trace_every_iter=1, tol=1e-30,
                         check_every=ce)
    merit = r.iter_trace[:, 0]  # merit of iteration k (1-based) at index k - 1
    alone = {1: 0, 2: 0, 3: 0}
    prev_check = None
    for row in r.trace[:-1]:
        k, t = int(row[C["k"]]), int(row[C["t"]])
        ks = k - t                             # iterations done when this outer loop began
        m0 = merit[ks]                         # R~_{r,0}: the loop's first iteration
        mp = merit[prev_check - 1] if prev_check is not None and prev_check > ks else m0
        mk = merit[k - 1]
        assert row[C["merit"]] == mk and row[C["merit0"]] == m0 and row[C["merit_prev"]] == mp
        c1 = mk <= 0.2 * m0
        c2 = mk <= 0.6 * m0 and mk > mp
        c3 = t >= 0.2 * k
        assert bool(row[C["restart"]]) == (c1 or c2 or c3), k
        if c1 + c2 + c3 == 1:
            alone[1 if c1 else 2 if c2 else 3] += 1
        prev_check = k
    return alone


def test_restart_criteria_bookkeeping(oracle_mod):
    """Criterion 1 alone fires on tiny; criterion 2 alone on a mixed-bounds LP checked every
    10 iterations; criterion 3 alone at the first check of both."""
    a = _criteria_pin(oracle_mod, lpgen.make("tiny"), 6000)
    b = _criteria_pin(oracle_mod, lpgen.mixed_bounds_lp(20, 20, 60, 0.15, seed=2), 3000, ce=10)
    assert a[3] >= 1 and b[3] >= 1
    assert a[1] + b[1] >= 1 and a[2] + b[2] >= 1, (a, b)


def test_halpern_weight_at_t0(oracle_mod):
    """w^{0,1} = w^{0,0}/2 + w_hat/2 with w^{0,0} = 0 (Algorithm 2, t = 0): half of the plain
    iteration's w_hat from the origin."""
    lp = lpgen.make("tiny")
    h = oracle_mod.solve(lp, max_iter=1, lambda_override=0.9)
    p = oracle_mod.solve(lp, max_iter=1, lambda_override=0.9, use_halpern=0)
    np.testing.assert_allclose(h.x_cur, 0.5 * p.x_cur, rtol=1e-14, atol=1e-300)
    np.testing.assert_allclose(h.y_cur, 0.5 * p.y_cur, rtol=1e-14, atol=1e-300)
    assert np.linalg.norm(p.x_cur) > 0 and np.linalg.norm(p.y_cur) > 0


@pytest.mark.parametrize("seed", [1, 2, 3])
def test_every_bound_kind_matches_certificate_and_highs(oracle_mod, seed):
    from scipy.optimize import linprog
    lp = lpgen.mixed_bounds_lp(20, 20, 60, 0.15, seed=seed)
    fl, fu = np.isfinite(lp.l), np.isfinite(lp.u)
    assert (lp.l == lp.u).any() and (fl & ~fu).any() and (~fl & fu).any() and (~fl & ~fu).any()
    r = oracle_mod.solve(lp)
    assert r.status == "OPTIMAL"
    A = lp.dense()
    hs = linprog(lp.c, A_ub=-A[lp.m1:], b_ub=-lp.b[lp.m1:], A_eq=A[:lp.m1], b_eq=lp.b[:lp.m1],
                 bounds=list(zip(np.where(fl, lp.l, None), np.where(fu, lp.u, None))),
                 method="highs")
    assert hs.status == 0
    for ref in (lp.cert.obj, hs.fun):
        assert abs(r.pobj - ref) <= 1e-7 * (1 + abs(ref))
    # x_bar in the box, fixed columns exactly at their value
    assert np.all(r.x >= lp.l - 1e-9) and np.all(r.x <= lp.u + 1e-9)
    fixed = lp.l == lp.u
    np.testing.assert_allclose(r.x[fixed], lp.l[fixed], rtol=1e-14)


def test_openmp_build_is_bit_identical(oracle_mod):
    for lp in (lpgen.make("tiny"), lpgen.mixed_bounds_lp(20, 20, 60, 0.15, seed=1),
               lpgen.make("zipf1m", scale=0.002)):
        a = oracle_mod.solve(lp, max_iter=700)
        b = oracle_mod.solve(lp, max_iter=700, threads=4)
        assert a.iters == b.iters and a.lam == b.lam
        for u, v in ((a.x, b.x), (a.y, b.y), (a.z, b.z), (a.x_cur, b.x_cur), (a.trace, b.trace)):
            np.testing.assert_array_equal(u, v)
