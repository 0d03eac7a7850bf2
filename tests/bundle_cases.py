"""Inputs with row bundles (runs of equal-length rows, and the shift-structured runs the
default finds) and an independent count of the bundle work items the library should build
for them.  Shared by the CPU schedule tests and the GPU parity tests."""
import numpy as np

import lpgen


def transport():
    # 70 demand rows of 300 nonzeros: one bundle of 64 rows and one of 6, 300 = 4 * 64 + 44
    return lpgen.transport_lp(300, 70, seed=601)


def ot():
    # 299 demand rows of 300 (columns renumbered: the last sink's columns move to the end)
    return lpgen.ot_lp(300, 300, seed=602)


def dense(seed=603, m1=150, m2=150, n=400):
    # every row of A has n nonzeros and every row of A^T m: runs in both matrices
    return lpgen.bernoulli_lp(m1, m2, n, 1.0, seed=seed)


def edge_lp(seed=620):
    """Shifted runs at the edges of the bundle rules: 65 equality rows of exactly 256
    nonzeros (one bundle of 64, the 65th row left to a tile), 2 equality rows of 300 (the
    smallest bundle), 40 random short equality rows, then 70 shifted inequality rows of 257
    (Pi_+ in the bundle finisher); columns boxed in [0, 10]."""
    rng = np.random.default_rng(seed)
    n = 40000
    rows = []
    rows += [r + 70 * np.arange(256) for r in range(65)]
    rows += [20000 + r + 60 * np.arange(300) for r in range(2)]
    rows += [np.sort(rng.choice(n, size=rng.integers(5, 30), replace=False)) for _ in range(40)]
    m1 = len(rows)
    rows += [100 + r + 150 * np.arange(257) for r in range(70)]
    rowptr = np.concatenate([[0], np.cumsum([len(c) for c in rows])]).astype(np.int64)
    colidx = np.concatenate(rows).astype(np.int32)
    val = rng.standard_normal(len(colidx)).astype(np.float32).astype(np.float64)
    m = len(rows)
    x0 = rng.uniform(0.0, 10.0, n)
    A = np.zeros(m)
    for i in range(m):
        A[i] = val[rowptr[i]:rowptr[i + 1]] @ x0[colidx[rowptr[i]:rowptr[i + 1]]]
    b = A.copy()
    b[m1:] -= 1.0
    c = rng.standard_normal(n)
    return lpgen.LP("bundle_edges", m1, m - m1, n, rowptr, colidx, val, b, c, np.zeros(n),
                    np.full(n, 10.0))


def expected_shifted_bundles(lp, min_len=16, max_len=16384):
    """Bundles (one work item each when rows have <= 64 entries) of the maximal runs of
    consecutive equal-length rows whose columns are, entry by entry, the previous row's plus
    one, cut into pieces of at most 64 rows, a last piece of one row left out."""
    rp, ci = lp.rowptr, lp.colidx
    lens = np.diff(rp)
    items, r = 0, 0
    while r < lp.m:
        L, e = lens[r], r + 1
        if min_len <= L <= max_len:
            while e < lp.m and lens[e] == L and np.array_equal(
                    ci[rp[e]:rp[e + 1]], ci[rp[e - 1]:rp[e]] + 1):
                e += 1
        full, rest = divmod(e - r, 64)
        items += (full + (rest >= 2)) * -(-L // 64)
        r = e
    return items
