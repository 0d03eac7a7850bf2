"""Host logic of the schedules (CPU): the row bundles hprlp_create would build, through the
host-only hprlp_plan_schedule, against an independent count from the matrix itself, on
LPs whose row runs are shift-structured (transportation demand rows, optimal-transport
demand rows, QAP rows of N + 1, edge cases), random LPs (none), forced bundles of every
equal-length run (dense LPs, both matrices), and the refusals."""
import numpy as np
import pytest

import lpgen
from bundle_cases import dense, edge_lp, expected_shifted_bundles, ot, transport
from paper_2408_12179_amd import hprlp


@pytest.fixture(scope="module")
def lib():
    return hprlp.load()


def expected_equal_run_bundles(lens, min_len=256, max_len=16384):
    """Forced bundles: maximal runs of equal lengths in [min_len, max_len], pieces of at
    most 64 rows, a last piece of one row left out; ceil(L / 64) work items per bundle."""
    items, r = 0, 0
    while r < len(lens):
        L, e = lens[r], r + 1
        if min_len <= L <= max_len:
            while e < len(lens) and lens[e] == L:
                e += 1
        full, rest = divmod(e - r, 64)
        items += (full + (rest >= 2)) * -(-int(L) // 64)
        r = e
    return items


def col_counts(lp, reorder=True):
    deg = np.bincount(lp.colidx, minlength=lp.n)
    return np.sort(deg)[::-1] if reorder else deg


CASES = {"transport": transport, "ot": ot, "qap20": lambda: lpgen.qap_lp(20, seed=1),
         "edges": edge_lp}


@pytest.mark.parametrize("name", list(CASES))
def test_default_bundles_shifted_runs_of_A(lib, name):
    lp = CASES[name]()
    a, t = hprlp.plan_schedule(lp, 0), hprlp.plan_schedule(lp, 1)
    assert a["bundle_items"] == expected_shifted_bundles(lp) > 0, (name, a)
    assert t["bundle_items"] == 0
    assert a["tiles"] + a["row_items"] + a["chunks"] + a["bundle_items"] <= a["items"]
    off = hprlp.plan_schedule(lp, 0, bundle_rows=0)
    assert off["bundle_items"] == 0 and off["items"] != a["items"]


@pytest.mark.parametrize("lp", [lpgen.bernoulli_lp(200, 200, 800, 0.05, seed=5),
                                lpgen.zipf_lp(3000, 3000, 12000, seed=6), dense()],
                         ids=["bernoulli", "zipf", "dense"])
def test_random_rows_get_no_bundles_by_default(lib, lp):
    assert hprlp.plan_schedule(lp, 0)["bundle_items"] == 0
    assert hprlp.plan_schedule(lp, 1)["bundle_items"] == 0


def test_forced_bundles_every_equal_run(lib):
    lp = dense()   # 300 rows of 400, 400 columns of 300
    a = hprlp.plan_schedule(lp, 0, bundle_rows=1)
    t = hprlp.plan_schedule(lp, 1, bundle_rows=1)
    assert a["bundle_items"] == expected_equal_run_bundles(np.diff(lp.rowptr)) == 35
    assert t["bundle_items"] == expected_equal_run_bundles(col_counts(lp)) == 35
    assert a["tiles"] == a["row_items"] == a["chunks"] == 0       # every row is bundled
    # a transportation LP: A's demand rows (70 of 300) are bundled, A^T's columns of 2 are not
    lp = transport()
    a = hprlp.plan_schedule(lp, 0, bundle_rows=1)
    assert a["bundle_items"] == expected_equal_run_bundles(np.diff(lp.rowptr)) == 10
    assert hprlp.plan_schedule(lp, 1, bundle_rows=1)["bundle_items"] == 0


def test_bundles_keep_their_rows_under_any_schedule_parameters(lib):
    # bundle membership is fixed: tile shapes and split lengths change only the rest
    lp = edge_lp()
    want = expected_shifted_bundles(lp)
    for p in (dict(tile_nnz=256, tile_rows=64, short_max=16, split_len=64, chunk_nnz=256),
              dict(tile_nnz=2048, tile_rows=1024, short_max=2048, split_len=65536, chunk_nnz=8192)):
        assert hprlp.plan_schedule(lp, 0, **p)["bundle_items"] == want


def test_plan_schedule_refusals(lib):
    lp = transport()
    with pytest.raises(hprlp.HPRLPError) as e:
        hprlp.plan_schedule(lp, 0, bundle_rows=1, t1_zero=1)
    assert e.value.code == hprlp.EINVAL
    with pytest.raises(hprlp.HPRLPError) as e:
        hprlp.plan_schedule(lp, 2)
    assert e.value.code == hprlp.EINVAL
    bad = lpgen.transport_lp(30, 20, seed=1)
    bad.colidx = bad.colidx.copy()
    bad.colidx[5] = bad.n      # out of range
    with pytest.raises(hprlp.HPRLPError) as e:
        hprlp.plan_schedule(bad, 0)
    assert e.value.code == hprlp.EINVAL


def composed_lp(seed):
    """Rows from random segments: random short rows, shift-structured runs (columns of row
    r + 1 = row r's plus one) and equal-length runs with random columns, of random lengths
    (8..600) and run sizes (1..150), in a random order."""
    rng = np.random.default_rng(seed)
    n = 200000
    rows = []
    for _ in range(rng.integers(5, 15)):
        kind = rng.integers(0, 3)
        R = int(rng.integers(1, 150))
        L = int(rng.choice([8, 15, 16, 17, 40, 64, 65, 200, 255, 256, 257, 600]))
        if kind == 0:
            rows += [np.sort(rng.choice(n, size=rng.integers(1, 30), replace=False)) for _ in range(R)]
        elif kind == 1:
            stride = int(rng.integers(R + 1, (n - R) // L))
            base = int(rng.integers(0, n - R - stride * (L - 1)))
            rows += [base + r + stride * np.arange(L) for r in range(R)]
        else:
            rows += [np.sort(rng.choice(n, size=L, replace=False)) for _ in range(R)]
    rowptr = np.concatenate([[0], np.cumsum([len(c) for c in rows])]).astype(np.int64)
    colidx = np.concatenate(rows).astype(np.int32)
    m = len(rows)
    return lpgen.LP("composed", m, 0, n, rowptr, colidx, np.ones(len(colidx)), np.ones(m),
                    np.ones(n), np.zeros(n), np.full(n, 1.0))


@pytest.mark.parametrize("seed", range(12))
def test_bundle_detection_on_composed_matrices(lib, seed):
    lp = composed_lp(seed)
    assert hprlp.plan_schedule(lp, 0)["bundle_items"] == expected_shifted_bundles(lp)
    assert hprlp.plan_schedule(lp, 0, bundle_rows=1)["bundle_items"] == \
        expected_equal_run_bundles(np.diff(lp.rowptr))
    assert hprlp.plan_schedule(lp, 1, bundle_rows=1)["bundle_items"] == \
        expected_equal_run_bundles(col_counts(lp))
    assert hprlp.plan_schedule(lp, 0, bundle_rows=0)["bundle_items"] == 0
