"""Seeded synthetic LP generators shared by the oracle tests, the GPU tests and the benchmark.

This module draws problem data only.  It holds none of the HPR-LP arithmetic: no scaling,
no iteration, no residuals.  Every problem has the form of the paper's primal LP (Section 1,
eq. primalLP):

    min <c, x>  s.t.  A1 x = b1,  A2 x >= b2,  l <= x <= u,

stored as one CSR matrix A = [A1; A2] (m1 equality rows first, then m2 inequality rows).

Where a KKT certificate is built, it is built by construction: a primal point x0 in the box,
a dual point y0 in D = R^m1 x R^m2_+, and a reduced cost z0 complementary to x0 are drawn
first; then b is set from x0 (slack on the loose inequality rows) and c := A^T y0 + z0.  The
triple then satisfies the KKT system (Section 2, eq. KKT) and the optimal value is <c, x0>.

Random streams: numpy PCG64 (``default_rng``) with base seed 240812179; workload k uses
base + k, instance i of the batched workload uses base + 1000 + i.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np

BASE_SEED = 240812179


@dataclass
class Certificate:
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    obj: float  # <c, x0>, the exact optimal value up to the rounding of b and c


@dataclass
class LP:
    name: str
    m1: int
    m2: int
    n: int
    rowptr: np.ndarray  # int64 [m+1]
    colidx: np.ndarray  # int32 [nnz]
    val: np.ndarray     # float64 [nnz], every value exactly representable in float32
    b: np.ndarray
    c: np.ndarray
    l: np.ndarray
    u: np.ndarray
    cert: Optional[Certificate] = None
    # batched workloads: instance boundaries (row and column offsets, per-instance m1)
    inst_row_off: Optional[np.ndarray] = None
    inst_col_off: Optional[np.ndarray] = None
    inst_m1: Optional[np.ndarray] = None
    meta: dict = field(default_factory=dict)

    @property
    def m(self) -> int:
        return self.m1 + self.m2

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])

    def eq_mask(self) -> np.ndarray:
        """True for equality rows (A1), False for inequality rows (A2).  Inside a batched
        workload each instance keeps its own [A1_i; A2_i] order."""
        mask = np.zeros(self.m, dtype=bool)
        if self.inst_row_off is None:
            mask[:self.m1] = True
        else:
            for r0, m1 in zip(self.inst_row_off[:-1], self.inst_m1):
                mask[r0:r0 + m1] = True
        return mask

    def dense(self) -> np.ndarray:
        A = np.zeros((self.m, self.n))
        for i in range(self.m):
            s, e = self.rowptr[i], self.rowptr[i + 1]
            A[i, self.colidx[s:e]] = self.val[s:e]
        return A

    def instance(self, i: int) -> "LP":
        """Extract instance i of a batched (block-diagonal) workload as a standalone LP."""
        assert self.inst_row_off is not None
        r0, r1 = int(self.inst_row_off[i]), int(self.inst_row_off[i + 1])
        c0, c1 = int(self.inst_col_off[i]), int(self.inst_col_off[i + 1])
        s, e = int(self.rowptr[r0]), int(self.rowptr[r1])
        cert = None
        if self.cert is not None:
            x, y, z = self.cert.x[c0:c1], self.cert.y[r0:r1], self.cert.z[c0:c1]
            cert = Certificate(x, y, z, float(np.dot(self.c[c0:c1], x)))
        m1 = int(self.inst_m1[i])
        return LP(f"{self.name}[{i}]", m1, (r1 - r0) - m1, c1 - c0,
                  (self.rowptr[r0:r1 + 1] - s).astype(np.int64),
                  (self.colidx[s:e] - c0).astype(np.int32), self.val[s:e].copy(),
                  self.b[r0:r1].copy(), self.c[c0:c1].copy(), self.l[c0:c1].copy(),
                  self.u[c0:c1].copy(), cert)


# --------------------------------------------------------------------------------------
# building blocks
# --------------------------------------------------------------------------------------

def _fp32_normal(rng: np.random.Generator, k: int) -> np.ndarray:
    """N(0,1) values rounded to float32 (so FP32 storage of A is lossless); no exact zeros."""
    v = rng.standard_normal(k).astype(np.float32)
    bad = v == 0
    while bad.any():
        v[bad] = rng.standard_normal(int(bad.sum())).astype(np.float32)
        bad = v == 0
    return v.astype(np.float64)


def _rows_from_lengths(lengths: np.ndarray) -> np.ndarray:
    rowptr = np.zeros(len(lengths) + 1, dtype=np.int64)
    np.cumsum(lengths, out=rowptr[1:])
    return rowptr


def _dedupe_rows(rowptr: np.ndarray, col: np.ndarray, draw, n: int) -> np.ndarray:
    """Redraw repeated column indices within a row until every row's columns are distinct,
    then sort each row's columns ascending.  ``draw(k)`` returns k fresh column indices."""
    m = len(rowptr) - 1
    row_of = np.repeat(np.arange(m, dtype=np.int64), np.diff(rowptr))
    pending = np.arange(len(col), dtype=np.int64)  # entry positions still to be checked
    while len(pending):
        key = row_of[pending] * n + col[pending]
        order = np.argsort(key, kind="stable")
        ks = key[order]
        dup = np.zeros(len(ks), dtype=bool)
        dup[1:] = ks[1:] == ks[:-1]
        if not dup.any():
            break
        redo = pending[order[dup]]
        col[redo] = draw(len(redo))
        # only rows that had a repeat need checking again
        bad_rows = np.unique(row_of[redo])
        mask = np.zeros(m, dtype=bool)
        mask[bad_rows] = True
        pending = np.nonzero(mask[row_of])[0]
    key = row_of * n + col
    order = np.argsort(key, kind="stable")
    return col[order]


def _certificate(rng, A_rowptr, A_col, A_val, m1, m2, n, l, u, boxed_tie="thirds"):
    """Draw a KKT point (x0, y0, z0) and derive b and c from it."""
    m = m1 + m2
    x0 = np.empty(n)
    z0 = np.zeros(n)
    fl, fu = np.isfinite(l), np.isfinite(u)
    boxed = fl & fu
    lower_only = fl & ~fu
    upper_only = ~fl & fu
    free = ~fl & ~fu
    # boxed: at l w.p. 1/3, at u w.p. 1/3, else uniform inside
    k = int(boxed.sum())
    r = rng.random(k)
    lb, ub = l[boxed], u[boxed]
    xb = lb + rng.random(k) * (ub - lb)
    zb = np.zeros(k)
    at_l = r < 1 / 3
    at_u = (r >= 1 / 3) & (r < 2 / 3)
    xb[at_l] = lb[at_l]
    xb[at_u] = ub[at_u]
    zb[at_l] = rng.exponential(1.0, int(at_l.sum()))
    zb[at_u] = -rng.exponential(1.0, int(at_u.sum()))
    x0[boxed], z0[boxed] = xb, zb
    # [l, inf): at l w.p. 1/2 else l + U(0, 10)
    k = int(lower_only.sum())
    at = rng.random(k) < 0.5
    xl = l[lower_only] + np.where(at, 0.0, rng.random(k) * 10.0)
    zl = np.where(at, rng.exponential(1.0, k), 0.0)
    x0[lower_only], z0[lower_only] = xl, zl
    # (-inf, u]: mirror image
    k = int(upper_only.sum())
    at = rng.random(k) < 0.5
    x0[upper_only] = u[upper_only] - np.where(at, 0.0, rng.random(k) * 10.0)
    z0[upper_only] = np.where(at, -rng.exponential(1.0, k), 0.0)
    # free: U(-10, 10), z0 = 0
    k = int(free.sum())
    x0[free] = rng.uniform(-10.0, 10.0, k)

    y0 = np.zeros(m)
    y0[:m1] = rng.standard_normal(m1)
    tight = rng.random(m2) < 0.5
    slack = np.where(tight, 0.0, rng.uniform(0.1, 10.0, m2))
    y0[m1:] = np.where(tight, rng.exponential(1.0, m2), 0.0)

    Ax = _csr_matvec(A_rowptr, A_col, A_val, x0, m)
    b = Ax.copy()
    b[m1:] -= slack
    c = _csr_rmatvec(A_rowptr, A_col, A_val, y0, n) + z0
    return b, c, Certificate(x0, y0, z0, float(np.dot(c, x0)))


def _csr_matvec(rowptr, col, val, x, m):
    row_of = np.repeat(np.arange(m), np.diff(rowptr))
    return np.bincount(row_of, weights=val * x[col], minlength=m).astype(np.float64)


def _csr_rmatvec(rowptr, col, val, y, n):
    row_of = np.repeat(np.arange(len(rowptr) - 1), np.diff(rowptr))
    return np.bincount(col, weights=val * y[row_of], minlength=n).astype(np.float64)


# --------------------------------------------------------------------------------------
# workload families
# --------------------------------------------------------------------------------------

def bernoulli_lp(m1: int, m2: int, n: int, density: float, seed: int, name="bernoulli",
                 half_boxed=True) -> LP:
    """Random sparse LP with an i.i.d. Bernoulli(density) pattern and N(0,1) (FP32-exact)
    values; l = 0, u = 10 on a seeded half of the columns and +inf on the rest."""
    rng = np.random.default_rng(seed)
    m = m1 + m2
    lengths = rng.binomial(n, density, size=m).astype(np.int64)
    rowptr = _rows_from_lengths(lengths)
    nnz = int(rowptr[-1])
    col = rng.integers(0, n, size=nnz).astype(np.int64)
    col = _dedupe_rows(rowptr, col, lambda k: rng.integers(0, n, size=k), n)
    val = _fp32_normal(rng, nnz)
    l = np.zeros(n)
    u = np.full(n, np.inf)
    if half_boxed:
        boxed = rng.permutation(n)[: n // 2]
        u[boxed] = 10.0
    b, c, cert = _certificate(rng, rowptr, col, val, m1, m2, n, l, u)
    return LP(name, m1, m2, n, rowptr, col.astype(np.int32), val, b, c, l, u, cert,
              meta=dict(family="bernoulli", density=density, seed=seed))


def mixed_bounds_lp(m1: int, m2: int, n: int, density: float, seed: int,
                    name="mixed_bounds") -> LP:
    """Bernoulli LP whose columns take every kind of bound, in equal shares: boxed
    [l, u] (l ~ U(-5, 0), u = l + U(1, 10)), fixed l = u ~ U(-3, 3), lower-only [l, +inf),
    upper-only (-inf, u] and free.  Certificate as for bernoulli_lp (a fixed column is a box
    of width 0: x0 = l = u with any sign of z0)."""
    rng = np.random.default_rng(seed)
    m = m1 + m2
    lengths = rng.binomial(n, density, size=m).astype(np.int64)
    rowptr = _rows_from_lengths(lengths)
    nnz = int(rowptr[-1])
    col = rng.integers(0, n, size=nnz).astype(np.int64)
    col = _dedupe_rows(rowptr, col, lambda k: rng.integers(0, n, size=k), n)
    val = _fp32_normal(rng, nnz)
    kind = rng.integers(0, 5, size=n)
    lo = rng.uniform(-5.0, 0.0, n)
    width = rng.uniform(1.0, 10.0, n)
    fix = rng.uniform(-3.0, 3.0, n)
    l = np.select([kind == 0, kind == 1, kind == 2], [lo, fix, lo], -np.inf)
    u = np.select([kind == 0, kind == 1, kind == 3], [lo + width, fix, lo + width], np.inf)
    b, c, cert = _certificate(rng, rowptr, col, val, m1, m2, n, l, u)
    return LP(name, m1, m2, n, rowptr, col.astype(np.int32), val, b, c, l, u, cert,
              meta=dict(family="mixed_bounds", density=density, seed=seed))


def zipf_lp(m1: int, m2: int, n: int, seed: int, row_len=(5, 40), zipf_s=1.1,
            free_frac=0.3, ub_range=(1.0, 100.0), name="zipf") -> LP:
    """Large sparse LP: row lengths U{row_len}, columns drawn from a bounded Zipf(zipf_s)
    popularity over a seeded column permutation (no repeats within a row), values N(0,1)
    in FP32-exact form; free_frac of the columns free, the rest boxed in [0, U_j] with
    U_j ~ U(ub_range)."""
    rng = np.random.default_rng(seed)
    m = m1 + m2
    lengths = rng.integers(row_len[0], row_len[1] + 1, size=m).astype(np.int64)
    rowptr = _rows_from_lengths(lengths)
    nnz = int(rowptr[-1])
    ranks = np.arange(1, n + 1, dtype=np.float64)
    cdf = np.cumsum(ranks ** (-zipf_s))
    cdf /= cdf[-1]
    perm = rng.permutation(n).astype(np.int64)

    def draw(k):
        r = np.searchsorted(cdf, rng.random(k), side="right")
        return perm[np.minimum(r, n - 1)]

    col = draw(nnz)
    col = _dedupe_rows(rowptr, col, draw, n)
    val = _fp32_normal(rng, nnz)
    l = np.zeros(n)
    u = rng.uniform(ub_range[0], ub_range[1], n)
    free = rng.random(n) < free_frac
    l[free] = -np.inf
    u[free] = np.inf
    b, c, cert = _certificate(rng, rowptr, col, val, m1, m2, n, l, u)
    return LP(name, m1, m2, n, rowptr, col.astype(np.int32), val, b, c, l, u, cert,
              meta=dict(family="zipf", zipf_s=zipf_s, row_len=row_len, seed=seed))


def transport_lp(n_src: int, n_dst: int, seed: int, name="transport") -> LP:
    """Transportation LP: flow x_ij at column i*n_dst + j; n_src equality supply rows
    (sum_j x_ij = s_i), then n_dst inequality demand rows (sum_i x_ij >= d_j); all
    coefficients 1; costs U(1,100) rounded to FP32; integer s, d ~ U{10..1000} with every
    supply multiplied by ceil(sum d / sum s) so total supply covers total demand; x >= 0."""
    rng = np.random.default_rng(seed)
    n = n_src * n_dst
    sup = rng.integers(10, 1001, size=n_src).astype(np.float64)
    dem = rng.integers(10, 1001, size=n_dst).astype(np.float64)
    k = max(1.0, float(np.ceil(dem.sum() / sup.sum())))
    sup *= k
    cost = rng.uniform(1.0, 100.0, n).astype(np.float32).astype(np.float64)
    sup_rowptr = np.arange(n_src + 1, dtype=np.int64) * n_dst
    dem_rowptr = n + np.arange(n_dst + 1, dtype=np.int64) * n_src
    rowptr = np.concatenate([sup_rowptr, dem_rowptr[1:]])
    sup_cols = np.arange(n, dtype=np.int64)
    dem_cols = (np.arange(n_src, dtype=np.int64)[None, :] * n_dst
                + np.arange(n_dst, dtype=np.int64)[:, None]).ravel()
    col = np.concatenate([sup_cols, dem_cols]).astype(np.int32)
    val = np.ones(2 * n)
    b = np.concatenate([sup, dem])
    return LP(name, n_src, n_dst, n, rowptr, col, val, b, cost, np.zeros(n),
              np.full(n, np.inf), None,
              meta=dict(family="transport", n_src=n_src, n_dst=n_dst, seed=seed,
                        supply_factor=k))


def ot_lp(n_src: int, n_dst: int, seed: int, name="ot") -> LP:
    """Balanced optimal-transport LP, every row an equality: flow x_ij at column
    i n_dst + j, supply rows sum_j x_ij = s_i for every i, then demand rows sum_i x_ij = d_j
    for j < n_dst - 1 (the last one follows from the others, so A has full row rank).
    Sources and sinks are uniform points in the unit square; cost 100 |p_i - q_j|^2 rounded
    to FP32; integer weights U{1..100}, supplies scaled by the total demand and demands by
    the total supply so both sum to the same value; x >= 0."""
    rng = np.random.default_rng(seed)
    p, q = rng.random((n_src, 2)), rng.random((n_dst, 2))
    sw = rng.integers(1, 101, n_src).astype(np.float64)
    dw = rng.integers(1, 101, n_dst).astype(np.float64)
    sup, dem = sw * dw.sum(), dw * sw.sum()
    n = n_src * n_dst
    cost = (100.0 * ((p[:, None, :] - q[None, :, :]) ** 2).sum(-1)).ravel()
    cost = cost.astype(np.float32).astype(np.float64)
    nd = n_dst - 1
    sup_rowptr = np.arange(n_src + 1, dtype=np.int64) * n_dst
    dem_rowptr = n + np.arange(nd + 1, dtype=np.int64) * n_src
    rowptr = np.concatenate([sup_rowptr, dem_rowptr[1:]])
    sup_cols = np.arange(n, dtype=np.int64)
    dem_cols = (np.arange(n_src, dtype=np.int64)[None, :] * n_dst
                + np.arange(nd, dtype=np.int64)[:, None]).ravel()
    col = np.concatenate([sup_cols, dem_cols]).astype(np.int32)
    m = n_src + nd
    return LP(name, m, 0, n, rowptr, col, np.ones(len(col)), np.concatenate([sup, dem[:nd]]),
              cost, np.zeros(n), np.full(n, np.inf), None,
              meta=dict(family="ot", n_src=n_src, n_dst=n_dst, seed=seed))


def qap_lp(N: int, seed: int, name="qap") -> LP:
    """LP relaxation of a quadratic assignment problem, in the form of the paper's large QAP
    experiments (Section 4.4, Adams-Johnson linearisation), every index running over 1..N.

    Columns: s_ijkl >= 0 at ((i N + j) N + k) N + l, then 0 <= x_kl <= 1 at N^4 + k N + l.
    Equality rows, in this order:
      (a) sum_i s_ijkl - x_kl = 0  for every (j, k, l), row (j N + k) N + l
      (b) sum_j s_ijkl - x_kl = 0  for every (i, k, l), row N^3 + (i N + k) N + l
      (c) s_ijkl - s_klij = 0      for every pair p = i N + j < q = k N + l (q-major within p)
      (d) sum_j x_ij = 1 for every i, then (e) sum_i x_ij = 1 for every j.
    Cost a_ik b_jl on s_ijkl, 0 on x.  The flow matrix a and the distance matrix b are
    symmetric with zero diagonal and integer entries U{0..99}, like uniformly random QAPLIB
    instances (QAPLIB itself is not available); all data are exact in FP32.  No certificate:
    the optimal value is that of the relaxation."""
    rng = np.random.default_rng(seed)

    def sym():
        t = np.triu(rng.integers(0, 100, size=(N, N)), 1)
        return (t + t.T).astype(np.float64)

    flow, dist = sym(), sym()
    N2, N3, N4 = N * N, N ** 3, N ** 4
    ar = np.arange(N, dtype=np.int64)
    xcol = lambda k, l: N4 + k * N + l  # noqa: E731
    # (a): row (j, k, l) holds s_{i j k l} for i = 0..N-1, then x_kl
    j, k, l = np.meshgrid(ar, ar, ar, indexing="ij")
    j, k, l = j.ravel(), k.ravel(), l.ravel()
    s_a = ((ar[None, :] * N + j[:, None]) * N + k[:, None]) * N + l[:, None]
    cols_a = np.concatenate([s_a, xcol(k, l)[:, None]], axis=1)
    # (b): row (i, k, l) holds s_{i j k l} for j = 0..N-1, then x_kl
    i = j  # same (first, k, l) enumeration
    s_b = ((i[:, None] * N + ar[None, :]) * N + k[:, None]) * N + l[:, None]
    cols_b = np.concatenate([s_b, xcol(k, l)[:, None]], axis=1)
    vals_ab = np.concatenate([np.ones((N3, N)), -np.ones((N3, 1))], axis=1)
    # (c): pairs p < q
    p, q = np.triu_indices(N2, 1)
    cols_c = np.stack([p * N2 + q, q * N2 + p], axis=1)
    vals_c = np.tile(np.array([1.0, -1.0]), (len(p), 1))
    # (d), (e)
    cols_d = N4 + ar[:, None] * N + ar[None, :]
    cols_e = N4 + ar[None, :] * N + ar[:, None]
    colidx = np.concatenate([cols_a.ravel(), cols_b.ravel(), cols_c.ravel(), cols_d.ravel(),
                             cols_e.ravel()]).astype(np.int32)
    val = np.concatenate([vals_ab.ravel(), vals_ab.ravel(), vals_c.ravel(),
                          np.ones(2 * N2)])
    lens = np.concatenate([np.full(2 * N3, N + 1), np.full(len(p), 2), np.full(2 * N, N)])
    rowptr = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    m = len(lens)
    b = np.concatenate([np.zeros(m - 2 * N), np.ones(2 * N)])
    n = N4 + N2
    cost = np.zeros(n)
    cost[:N4] = (flow[:, None, :, None] * dist[None, :, None, :]).ravel()  # a_ik b_jl
    lo = np.zeros(n)
    up = np.concatenate([np.full(N4, np.inf), np.ones(N2)])
    return LP(name, m, 0, n, rowptr, colidx, val, b, cost, lo, up, None,
              meta=dict(family="qap", N=N, seed=seed, flow=flow, dist=dist))


def batched_lp(n_inst: int, m_range=(1000, 50000), rho_range=(8.0, 30.0),
               seed_base: int = BASE_SEED + 1000, name="batched") -> LP:
    """n_inst independent Bernoulli LPs (the tiny-workload generator) packed block-diagonally:
    instance i has m_i ~ U{m_range}, n_i = 2 m_i, mean row length rho_i ~ U(rho_range),
    pattern Bernoulli(rho_i / n_i), m1_i = floor(m_i / 2).  Instance i uses seed
    seed_base + i for all of its draws (sizes included)."""
    parts: List[LP] = []
    for i in range(n_inst):
        rng = np.random.default_rng(seed_base + i)
        mi = int(rng.integers(m_range[0], m_range[1] + 1))
        rho = float(rng.uniform(rho_range[0], rho_range[1]))
        ni = 2 * mi
        parts.append(bernoulli_lp(mi // 2, mi - mi // 2, ni, rho / ni,
                                  seed=int(rng.integers(0, 2**62)), name=f"{name}[{i}]"))
    return pack_block_diagonal(parts, name)


def pack_block_diagonal(parts: List[LP], name="batched") -> LP:
    """Pack independent LPs into one block-diagonal CSR (instance rows and columns contiguous;
    inside an instance its equality rows come first)."""
    row_off = np.zeros(len(parts) + 1, dtype=np.int64)
    col_off = np.zeros(len(parts) + 1, dtype=np.int64)
    nnz_off = np.zeros(len(parts) + 1, dtype=np.int64)
    for i, p in enumerate(parts):
        row_off[i + 1] = row_off[i] + p.m
        col_off[i + 1] = col_off[i] + p.n
        nnz_off[i + 1] = nnz_off[i] + p.nnz
    m, n, nnz = int(row_off[-1]), int(col_off[-1]), int(nnz_off[-1])
    rowptr = np.zeros(m + 1, dtype=np.int64)
    col = np.empty(nnz, dtype=np.int32)
    val = np.empty(nnz)
    b, y0 = np.empty(m), np.empty(m)
    c, l, u, x0, z0 = (np.empty(n) for _ in range(5))
    have_cert = all(p.cert is not None for p in parts)
    for i, p in enumerate(parts):
        r0, c0, s0 = row_off[i], col_off[i], nnz_off[i]
        rowptr[r0 + 1:r0 + p.m + 1] = p.rowptr[1:] + s0
        col[s0:s0 + p.nnz] = p.colidx + c0
        val[s0:s0 + p.nnz] = p.val
        b[r0:r0 + p.m] = p.b
        c[c0:c0 + p.n], l[c0:c0 + p.n], u[c0:c0 + p.n] = p.c, p.l, p.u
        if have_cert:
            x0[c0:c0 + p.n], z0[c0:c0 + p.n] = p.cert.x, p.cert.z
            y0[r0:r0 + p.m] = p.cert.y
    cert = Certificate(x0, y0, z0, float(np.dot(c, x0))) if have_cert else None
    m1 = np.array([p.m1 for p in parts], dtype=np.int64)
    # the packed matrix is not [A1; A2] globally: per-instance m1 drives the cone D
    return LP(name, int(m1.sum()), m - int(m1.sum()), n, rowptr, col, val, b, c, l, u, cert,
              inst_row_off=row_off, inst_col_off=col_off, inst_m1=m1,
              meta=dict(family="batched", n_inst=len(parts)))


def tiny_boxed_lp(m1: int, m2: int, n: int, seed: int, density=0.7) -> LP:
    """Very small LP with every column boxed (for exhaustive vertex enumeration): x in [l, u]
    with l ~ U(-3, 0), u = l + U(1, 5); A dense-ish N(0,1) FP32-exact; b from an interior
    point (slack on every inequality row), c ~ N(0,1) FP32-exact (no certificate)."""
    rng = np.random.default_rng(seed)
    m = m1 + m2
    mask = rng.random((m, n)) < density
    for i in range(m):  # no empty row
        if not mask[i].any():
            mask[i, rng.integers(0, n)] = True
    dense = np.where(mask, _fp32_normal(rng, m * n).reshape(m, n), 0.0)
    l = -rng.uniform(0.0, 3.0, n)
    u = l + rng.uniform(1.0, 5.0, n)
    xin = l + rng.uniform(0.2, 0.8, n) * (u - l)
    b = dense @ xin
    b[m1:] -= rng.uniform(0.1, 2.0, m2)
    c = _fp32_normal(rng, n)
    rowptr = _rows_from_lengths(mask.sum(axis=1))
    col = np.concatenate([np.nonzero(mask[i])[0] for i in range(m)]).astype(np.int32)
    val = dense[mask]
    return LP(f"tiny{seed}", m1, m2, n, rowptr, col, val, b, c, l, u, None,
              meta=dict(family="tiny", seed=seed))


# --------------------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------------------

WORKLOADS = {
    "tiny": "tiny random sparse LP: m1=50, m2=50, n=200, Bernoulli(0.05), plain FP64",
    "zipf1m": "single large sparse LP: m=500k (half equality), n=1M, row lengths U{5..40}, "
          "Zipf(1.1) columns, plain FP64",
    "zipf4m": "single larger sparse LP: m=2M, n=4M, same generator as zipf1m, FP32->FP64",
    "batch256": "batched: 256 Bernoulli LPs, m_i~U{1k..50k}, n_i=2m_i, 8-30 nnz/row",
    "transport10m": "transportation 2000 x 5000: n=10M, m=7000, FP32->FP64",
    "ot4m": "balanced optimal transport 2048 x 2048 (all equality rows, last demand row "
            "dropped): n=4.19M, m=4095, nnz=8.39M, plain FP64",
    "qap40": "QAP LP relaxation (Section 4.4 form), N=40 random symmetric flow/distance "
             "U{0..99}: n=2.56M, m=1.41M (all equality), nnz=7.81M, plain FP64",
}


def make(name: str, scale: float = 1.0) -> LP:
    """Build a named workload.  ``scale`` shrinks the large workloads (row and column counts)
    for tests that must finish in seconds; scale=1 gives the full size."""
    if name == "tiny":
        return bernoulli_lp(50, 50, 200, 0.05, seed=BASE_SEED + 0, name="tiny")
    if name in ("zipf1m", "zipf4m"):
        m = {"zipf1m": 500_000, "zipf4m": 2_000_000}[name]
        m = max(8, int(round(m * scale)))
        k = 1 if name == "zipf1m" else 2
        return zipf_lp(m // 2, m - m // 2, 2 * m, seed=BASE_SEED + k, name=name)
    if name == "batch256":
        n_inst = max(1, int(round(256 * scale))) if scale < 1 else 256
        mr = (1000, 50000) if scale >= 1 else (max(20, int(1000 * scale)),
                                                max(40, int(50000 * scale)))
        return batched_lp(n_inst, m_range=mr, name="batch256")
    if name == "transport10m":
        s = max(2, int(round(2000 * scale)))
        d = max(2, int(round(5000 * scale)))
        return transport_lp(s, d, seed=BASE_SEED + 4, name="transport10m")
    if name == "ot4m":
        k = max(2, int(round(2048 * scale ** 0.5)))
        return ot_lp(k, k, seed=BASE_SEED + 6, name="ot4m")
    if name == "qap40":  # scale acts on the nonzeros, which grow as N^4
        N = max(3, int(round(40 * scale ** 0.25)))
        return qap_lp(N, seed=BASE_SEED + 5, name="qap40")
    raise KeyError(name)
