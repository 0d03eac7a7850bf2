"""The C example (paper_2408_12179_amd/examples/solve_transport.c) uses the library from plain
C with a hipMalloc'ed workspace, no Python or torch in the process.  Its objective must match
the oracle's on the same 2 x 3 transportation LP."""
import os
import subprocess

import numpy as np
import pytest

import lpgen
import oracle

pytestmark = pytest.mark.gpu

EXE = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                   "paper_2408_12179_amd", "examples", "solve_transport")


def test_c_example_matches_oracle():
    assert os.path.exists(EXE), "build the library (it also builds the C example)"
    out = subprocess.run([EXE], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stderr
    line = out.stdout.split("\n")[0].split()
    status, pobj = int(line[1]), float(line[5])
    assert status == 1
    lp = lpgen.LP("transport2x3", 2, 3, 6, np.array([0, 3, 6, 8, 10, 12], dtype=np.int64),
                  np.array([0, 1, 2, 3, 4, 5, 0, 3, 1, 4, 2, 5], dtype=np.int32), np.ones(12),
                  np.array([20.0, 30, 10, 25, 15]), np.array([4.0, 6, 9, 5, 3, 8]),
                  np.zeros(6), np.full(6, np.inf))
    ref = oracle.solve(lp)
    assert ref.status == "OPTIMAL"
    assert abs(pobj - ref.pobj) <= 1e-7 * (1 + abs(ref.pobj)), (pobj, ref.pobj)
