"""The schedule autotuner: whatever schedules it picks, the iterates stay on the oracle's
(the schedule only changes the order of the sums, within the 1e-10 bar)."""
import numpy as np
import pytest

import lpgen
import oracle
from paper_2408_12179_amd import hprlp

pytestmark = pytest.mark.gpu


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a - b)


@pytest.mark.parametrize("name,scale", [("zipf1m", 0.02), ("transport10m", 0.1)])
def test_autotuned_iterate_parity(name, scale):
    lp = lpgen.make(name, scale)
    assert lp.nnz >= 100000  # large enough for the tuner to run
    ref = oracle.solve(lp, max_iter=100)
    s = hprlp.Solver(lp, max_iter=100, lambda_override=ref.lam, autotune=1)
    sa, st = s.schedule(0), s.schedule(1)
    print(name, "A:", sa, "A^T:", st)
    assert sa["tuned_ms"] > 0 and st["tuned_ms"] > 0
    sol = s.solve()
    for nm, a, b in (("x", sol.x, ref.x), ("y", sol.y, ref.y), ("z", sol.z, ref.z),
                     ("x_cur", s.iterate(hprlp.XCUR), ref.x_cur)):
        assert rel(a, b) <= 1e-10, (nm, rel(a, b))


def test_autotuned_batched_parity():
    lp = lpgen.batched_lp(12, m_range=(500, 3000), name="tune12")
    assert lp.nnz >= 100000
    iters = 200
    refs = [oracle.solve(lp.instance(i), max_iter=iters, check_every=100) for i in range(12)]
    s = hprlp.Solver(lp, batched=True, lambdas=[r.lam for r in refs], max_iter=iters,
                     check_every=100, autotune=1)
    print("A:", s.schedule(0), "A^T:", s.schedule(1))
    sol = s.solve()
    for i, ref in enumerate(refs):
        r0, r1 = lp.inst_row_off[i], lp.inst_row_off[i + 1]
        c0, c1 = lp.inst_col_off[i], lp.inst_col_off[i + 1]
        assert rel(sol.x[c0:c1], ref.x) <= 1e-10 and rel(sol.y[r0:r1], ref.y) <= 1e-10, i
