"""GPU parity on the inputs that pin SigmaUpdate's reset branch and every kind of column
bound (the CPU pins are in test_oracle_sigma_restart.py).

  * The four sigma := 1 cases of Algorithm 3 (Section 3.2): the first restart of the HIP path
    (host decision for one LP, k_decide on the device for a batch) sets sigma to exactly 1,
    like the oracle, and the iterates after 301 iterations (two restarts) agree with the
    oracle's to 1e-10 relative, norm-wise, and entry by entry to
    1e-10 (|ref_i| + 1e-3 ||ref||_inf).
  * Columns boxed, fixed (l = u), lower-only, upper-only and free (eq. update-x and
    delta*_C(-z) of Section 4.1): 100-iteration parity at the same bars, in FP64 and with A
    stored in FP32 (FP64_A32), single and batched, and full solves to rel. KKT 1e-8 with the
    objective within 1e-7 of the certificate (FP64 and MIXED).
"""
import numpy as np
import pytest

import lpgen
import oracle
from paper_2408_12179_amd import hprlp
from test_oracle_sigma_restart import sigma_cases

pytestmark = pytest.mark.gpu


def rel(a, b):
    d = np.linalg.norm(a - b)
    nb = np.linalg.norm(b)
    return d / nb if nb > 0 else d


def close_entrywise(a, b, tol=1e-10):
    scale = np.abs(b) + 1e-3 * (np.max(np.abs(b)) if b.size else 0.0)
    bad = np.abs(a - b) > tol * scale
    bad &= ~((a == 0) & (b == 0))
    assert not bad.any(), (np.flatnonzero(bad)[:5], a[bad][:5], b[bad][:5])


def _check_iterates(pairs):
    for name, a, b in pairs:
        assert rel(a, b) <= 1e-10, (name, rel(a, b))
        close_entrywise(a, b)


@pytest.mark.parametrize("case", range(4))
def test_sigma_reset_single(case):
    name, lp, s0 = sigma_cases()[case]
    ref = oracle.solve(lp, max_iter=301, sigma0=s0, tol=1e-30)
    s = hprlp.Solver(lp, max_iter=301, sigma0=s0, tol=1e-30, lambda_override=ref.lam)
    sol = s.solve()
    tr = s.trace()
    assert tr[0, 0] == 150 and tr[0, 16] == 1.0
    assert tr[0, 17] == 1.0 and ref.trace[0, 17] == 1.0, name
    np.testing.assert_array_equal(tr[:, 16], ref.trace[:, 16])
    _check_iterates([("x_bar", sol.x, ref.x), ("y_bar", sol.y, ref.y),
                     ("x_cur", s.iterate(hprlp.XCUR), ref.x_cur),
                     ("y_cur", s.iterate(hprlp.YCUR), ref.y_cur)])
    s.close()


@pytest.mark.parametrize("group", [(0, 1), (2,), (3,)], ids=["dx_dy_zero", "above", "below"])
def test_sigma_reset_batched(group):
    cases = [sigma_cases()[i] for i in group]
    s0 = cases[0][2]
    lp = lpgen.pack_block_diagonal([c[1] for c in cases], "sigma_reset")
    refs = [oracle.solve(c[1], max_iter=300, sigma0=s0, tol=1e-30, check_every=150)
            for c in cases]
    s = hprlp.Solver(lp, batched=True, lambdas=[r.lam for r in refs], max_iter=300,
                     sigma0=s0, tol=1e-30, check_every=150)
    sol = s.solve()
    for i, ref in enumerate(refs):
        tr = s.trace_instance(i)
        assert tr[0, 0] == 150 and tr[0, 8] == 1.0 and tr[0, 9] == 1.0, cases[i][0]
        r0, r1 = lp.inst_row_off[i], lp.inst_row_off[i + 1]
        c0, c1 = lp.inst_col_off[i], lp.inst_col_off[i + 1]
        _check_iterates([("x_bar", sol.x[c0:c1], ref.x), ("y_bar", sol.y[r0:r1], ref.y),
                         ("z_bar", sol.z[c0:c1], ref.z)])
    s.close()


@pytest.mark.parametrize("precision", [hprlp.FP64, hprlp.FP64_A32], ids=["fp64", "fp64a32"])
@pytest.mark.parametrize("seed", [1, 2])
def test_bound_kinds_iterate_parity(seed, precision):
    lp = lpgen.mixed_bounds_lp(40, 40, 120, 0.08, seed=seed)
    ref = oracle.solve(lp, max_iter=100)
    s = hprlp.Solver(lp, max_iter=100, lambda_override=ref.lam, precision=precision)
    sol = s.solve()
    _check_iterates([("x_bar", sol.x, ref.x), ("y_bar", sol.y, ref.y), ("z_bar", sol.z, ref.z),
                     ("x_cur", s.iterate(hprlp.XCUR), ref.x_cur),
                     ("y_cur", s.iterate(hprlp.YCUR), ref.y_cur)])
    # the box of width 0: x_bar is l~ exactly in the scaled space; unscaling (x = beta_b dc x~
    # with l~ = l / (dc beta_b)) rounds twice, so the original-space value is within 4 ulp
    fixed = lp.l == lp.u
    np.testing.assert_allclose(sol.x[fixed], lp.l[fixed], rtol=1e-15, atol=0)
    s.close()


def test_bound_kinds_batched_parity():
    parts = [lpgen.mixed_bounds_lp(40, 40, 120, 0.08, seed=s) for s in (1, 2, 3)]
    lp = lpgen.pack_block_diagonal(parts, "mixed_bounds3")
    refs = [oracle.solve(p, max_iter=300, check_every=100) for p in parts]
    s = hprlp.Solver(lp, batched=True, lambdas=[r.lam for r in refs], max_iter=300,
                     check_every=100)
    sol = s.solve()
    for i, ref in enumerate(refs):
        r0, r1 = lp.inst_row_off[i], lp.inst_row_off[i + 1]
        c0, c1 = lp.inst_col_off[i], lp.inst_col_off[i + 1]
        _check_iterates([("x_bar", sol.x[c0:c1], ref.x), ("y_bar", sol.y[r0:r1], ref.y),
                         ("z_bar", sol.z[c0:c1], ref.z)])
    s.close()


@pytest.mark.parametrize("precision", [hprlp.FP64, hprlp.MIXED], ids=["fp64", "mixed"])
def test_bound_kinds_full_solve(precision):
    lp = lpgen.mixed_bounds_lp(40, 40, 120, 0.08, seed=3)
    s = hprlp.Solver(lp, precision=precision)
    sol = s.solve()
    st = sol.stats
    assert sol.status == "OPTIMAL"
    assert abs(st["pobj"] - lp.cert.obj) <= 1e-7 * (1 + abs(lp.cert.obj))
    from lp_truth import relative_kkt
    assert max(relative_kkt(lp, sol.x, sol.y, sol.z)) <= 1.5e-8
    s.close()
