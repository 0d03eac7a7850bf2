"""The ablation variants of the paper's Section 4.2 (Fig. 1) as options, each against the
oracle running the same variant: relaxation rho (Step 9 of Algorithm 2; 1 = Douglas-
Rachford, 2 = Peaceman-Rachford), Halpern averaging on/off, restarts on/off, sigma update
on/off.  100-iteration iterates (and 700 iterations across restarts) at the 1e-10 bar."""
import numpy as np
import pytest

import lpgen
import oracle
from paper_2408_12179_amd import hprlp

pytestmark = pytest.mark.gpu

VARIANTS = {
    "DR": dict(rho=1.0, use_halpern=0, use_restart=0, sigma_update=0),
    "DR+restart+Halpern": dict(rho=1.0, use_halpern=1, use_restart=1, sigma_update=0),
    "DR+restart+Halpern+sigma": dict(rho=1.0, use_halpern=1, use_restart=1, sigma_update=1),
    "rho=1.6": dict(rho=1.6),
}


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


@pytest.mark.parametrize("variant", list(VARIANTS))
@pytest.mark.parametrize("name,scale,iters", [("tiny", 1, 700), ("zipf1m", 0.004, 100)])
def test_variant_parity(variant, name, scale, iters):
    lp = lpgen.make(name, scale)
    kw = VARIANTS[variant]
    ref = oracle.solve(lp, max_iter=iters, **kw)
    s = hprlp.Solver(lp, max_iter=iters, lambda_override=ref.lam, **kw)
    sol = s.solve()
    assert sol.stats["iters"] == ref.iters and sol.stats["restarts"] == ref.restarts
    for k, a, b in (("x", sol.x, ref.x), ("y", sol.y, ref.y), ("z", sol.z, ref.z),
                    ("x_cur", s.iterate(hprlp.XCUR), ref.x_cur),
                    ("y_cur", s.iterate(hprlp.YCUR), ref.y_cur)):
        assert rel(a, b) <= 1e-10, (variant, name, k, rel(a, b))


def test_relaxed_batched_and_mixed():
    # rho = 1 through the batched engine (device decisions, restart copies of x_rel) and
    # through the MIXED path (FP32 x_rel promoted)
    lp = lpgen.batched_lp(4, m_range=(30, 90), name="relax4")
    refs = [oracle.solve(lp.instance(i), max_iter=400, check_every=100, rho=1.0)
            for i in range(4)]
    s = hprlp.Solver(lp, batched=True, lambdas=[r.lam for r in refs], max_iter=400,
                     check_every=100, rho=1.0)
    sol = s.solve()
    for i, r in enumerate(refs):
        c0, c1 = lp.inst_col_off[i], lp.inst_col_off[i + 1]
        assert s.stats_instance(i)["restarts"] == r.restarts
        assert rel(sol.x[c0:c1], r.x) <= 1e-10, i
    tiny = lpgen.make("tiny")
    m = hprlp.Solver(tiny, precision=hprlp.MIXED, rho=1.0).solve()
    assert m.status == "OPTIMAL" and abs(m.stats["pobj"] - tiny.cert.obj) <= 1e-7 * (1 + abs(tiny.cert.obj))
