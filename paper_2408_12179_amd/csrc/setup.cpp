// Host-side preprocessing of the HPR-LP library: input validation, the preconditioning of
// Section 4.1 (Ruiz equilibration, a diagonal Pock-Chambolle pass with alpha = 1, b/c
// normalisation), the CSR transpose, and the row-length tile schedules of the SpMV passes.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "hprlp_setup.h"

namespace hprlp {

int validate_problem(int64_t m1, int64_t m2, int64_t n, const int64_t *rowptr,
                     const int32_t *colidx, const double *val, const double *b,
                     const double *c, const double *l, const double *u,
                     const hprlp_options &o, std::string &err) {
    if (!rowptr || !colidx || !val || !b || !c || !l || !u) {
        err = "null input pointer";
        return HPRLP_EINVAL;
    }
    if (m1 < 0 || m2 < 0 || m1 + m2 < 1 || n < 1 || m1 + m2 >= (1LL << 31) ||
        n >= (1LL << 31)) {
        err = "bad dimensions (need m1, m2 >= 0, m1 + m2 >= 1, n >= 1, both < 2^31)";
        return HPRLP_EDIM;
    }
    const int64_t m = m1 + m2;
    if (rowptr[0] != 0) {
        err = "rowptr[0] must be 0";
        return HPRLP_EDIM;
    }
    for (int64_t i = 0; i < m; ++i)
        if (rowptr[i + 1] < rowptr[i]) {
            err = "rowptr is not non-decreasing at row " + std::to_string(i);
            return HPRLP_EDIM;
        }
    const int64_t nnz = rowptr[m];
    if (nnz < 1 || nnz >= (1LL << 31)) {
        err = "nnz must be in [1, 2^31) (A must be non-zero)";
        return HPRLP_EDIM;
    }
    // A row whose columns strictly increase repeats none; only the other rows are checked
    // through a per-column marker (allocated on first need: a random access per nonzero
    // into an n-entry array is what this pass would otherwise cost).
    std::vector<int64_t> seen;
    for (int64_t i = 0; i < m; ++i) {
        bool increasing = true;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const int32_t j = colidx[p];
            if (j < 0 || j >= n) {
                err = "column index out of range in row " + std::to_string(i);
                return HPRLP_EDIM;
            }
            if (p > rowptr[i] && j <= colidx[p - 1]) increasing = false;
        }
        if (increasing) continue;
        if (seen.empty()) seen.assign((size_t)n, -1);
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const int32_t j = colidx[p];
            if (seen[j] == i) {
                err = "repeated column index in row " + std::to_string(i);
                return HPRLP_EDIM;
            }
            seen[j] = i;
        }
    }
    for (int64_t p = 0; p < nnz; ++p)
        if (!std::isfinite(val[p])) {
            err = "non-finite matrix value";
            return HPRLP_ENONFINITE;
        }
    for (int64_t i = 0; i < m; ++i)
        if (!std::isfinite(b[i])) {
            err = "non-finite b";
            return HPRLP_ENONFINITE;
        }
    for (int64_t j = 0; j < n; ++j) {
        if (!std::isfinite(c[j])) {
            err = "non-finite c";
            return HPRLP_ENONFINITE;
        }
        if (std::isnan(l[j]) || std::isnan(u[j])) {
            err = "NaN bound";
            return HPRLP_ENONFINITE;
        }
        if (l[j] > u[j] || l[j] == INFINITY || u[j] == -INFINITY) {
            err = "inconsistent bounds at column " + std::to_string(j);
            return HPRLP_EBOUNDS;
        }
    }
    if (o.precision != HPRLP_FP64)
        for (int64_t p = 0; p < nnz; ++p)
            if ((double)(float)val[p] != val[p]) {
                err = "FP32 storage of A needs every A value exactly representable in FP32";
                return HPRLP_ENOTLOSSLESS;
            }
    return HPRLP_OK;
}

int validate_options(const hprlp_options &o, std::string &err) {
    bool ok = o.tol > 0 && o.check_every >= 1 && o.max_iter >= 1 && o.alpha1 > 0 &&
              o.alpha1 < 1 && o.alpha2 > 0 && o.alpha2 < 1 && o.alpha3 > 0 && o.alpha3 < 1 &&
              o.sigma0 > 0 && o.ruiz_iters >= 0 && o.power_max_iter >= 1 && o.power_tol >= 0 &&
              (o.precision == HPRLP_FP64 || o.precision == HPRLP_MIXED ||
               o.precision == HPRLP_FP64_A32) && o.tol_switch > 0 &&
              o.tile_nnz >= 256 && o.tile_nnz <= kMaxTileNnz && o.tile_rows >= 1 &&
              o.tile_rows <= kMaxTileRows &&
              o.short_max >= 1 && o.short_max <= o.tile_nnz &&
              o.split_len >= o.short_max && o.chunk_nnz >= 256 && o.stall_ratio > 0 &&
              o.stall_ratio <= 1 && o.rho > 0 && o.rho <= 2 &&
              (o.t1_zero == 0 || o.t1_zero == 1) && (o.setup_on_host == 0 || o.setup_on_host == 1) &&
              o.tile_order >= -1 && o.tile_order <= 1 && !(o.t1_zero && o.tile_order == 1) &&
              o.bundle_rows >= -1 && o.bundle_rows <= 1 && !(o.t1_zero && o.bundle_rows == 1);
    if (!ok) err = "invalid option value";
    return ok ? HPRLP_OK : HPRLP_EINVAL;
}

void resolve_options(hprlp_options &o) {
    if (o.tile_nnz <= 0) o.tile_nnz = 2048;
    if (o.tile_rows <= 0) o.tile_rows = 512;
    if (o.short_max <= 0) o.short_max = 256;
    if (o.split_len <= 0) o.split_len = 8192;
    if (o.chunk_nnz <= 0) o.chunk_nnz = 4096;
    if (o.stall_ratio == 0) o.stall_ratio = 0.5;
    if (o.rho == 0) o.rho = 2.0;
}

// Transpose of a CSR matrix by counting sort over the column index.  pos[q] is the position
// in the original arrays of the q-th nonzero of the transpose (so any value array can be
// permuted later).  Rows of the transpose list their columns in increasing order.
void transpose(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *colidx,
               std::vector<int64_t> &rowptr_t, std::vector<int32_t> &colidx_t,
               std::vector<int32_t> &pos) {
    const int64_t nnz = rowptr[m];
    rowptr_t.assign((size_t)n + 1, 0);
    for (int64_t p = 0; p < nnz; ++p) rowptr_t[(size_t)colidx[p] + 1]++;
    for (int64_t j = 0; j < n; ++j) rowptr_t[j + 1] += rowptr_t[j];
    std::vector<int64_t> fill(rowptr_t.begin(), rowptr_t.end() - 1);
    colidx_t.resize((size_t)nnz);
    pos.resize((size_t)nnz);
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
            const int64_t q = fill[colidx[p]]++;
            colidx_t[q] = (int32_t)i;
            pos[q] = (int32_t)p;
        }
}

// Preconditioning of Section 4.1 on A~ = D_r A D_c.  Each pass computes row factors from the
// CSR rows and column factors from the rows of the transpose (same summation order as a
// row-by-row scan), then rescales both copies.  Ruiz: sqrt of the infinity norms; the
// Pock-Chambolle pass with alpha = 1: sqrt of the 1-norms.  Empty rows/columns keep 1.
void precondition(int64_t m, int64_t n, const int64_t *rowptr, const int32_t *colidx,
                  const std::vector<int64_t> &rowptr_t, const std::vector<int32_t> &pos,
                  const double *val, const hprlp_options &o, Scaling &s) {
    const int64_t nnz = rowptr[m];
    s.val.assign(val, val + nnz);
    std::vector<double> vt((size_t)nnz);
    for (int64_t q = 0; q < nnz; ++q) vt[q] = val[pos[q]];
    s.dr.assign((size_t)m, 1.0);
    s.dc.assign((size_t)n, 1.0);
    std::vector<double> rf((size_t)m), cf((size_t)n);
    const int passes = o.ruiz_iters + (o.pock_chambolle ? 1 : 0);
    for (int it = 0; it < passes; ++it) {
        const bool ruiz = it < o.ruiz_iters;
        for (int64_t i = 0; i < m; ++i) {
            double acc = 0.0;
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p) {
                const double a = std::fabs(s.val[p]);
                acc = ruiz ? std::max(acc, a) : acc + a;
            }
            rf[i] = acc > 0.0 ? std::sqrt(acc) : 1.0;
        }
        for (int64_t j = 0; j < n; ++j) {
            double acc = 0.0;
            for (int64_t q = rowptr_t[j]; q < rowptr_t[j + 1]; ++q) {
                const double a = std::fabs(vt[q]);
                acc = ruiz ? std::max(acc, a) : acc + a;
            }
            cf[j] = acc > 0.0 ? std::sqrt(acc) : 1.0;
        }
        for (int64_t i = 0; i < m; ++i)
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
                s.val[p] = s.val[p] / (rf[i] * cf[colidx[p]]);
        for (int64_t q = 0; q < nnz; ++q) vt[q] = s.val[pos[q]];
        for (int64_t i = 0; i < m; ++i) s.dr[i] = s.dr[i] / rf[i];
        for (int64_t j = 0; j < n; ++j) s.dc[j] = s.dc[j] / cf[j];
    }
}

void find_bundles(int64_t rows, const int64_t *rowptr, const int32_t *col,
                  const int32_t *inst_of_row, std::vector<Bundle> &out) {
    out.clear();
    auto len = [&](int64_t r) { return rowptr[r + 1] - rowptr[r]; };
    auto inst = [&](int64_t r) { return inst_of_row ? inst_of_row[r] : 0; };
    auto shifted = [&](int64_t a, int64_t b, int64_t L) {
        for (int64_t k : {(int64_t)0, L / 2, L - 1})
            if ((int64_t)col[rowptr[b] + k] != (int64_t)col[rowptr[a] + k] + 1) return false;
        return true;
    };
    const int64_t min_len = col ? kBundleMinShifted : kBundleMinLen;
    for (int64_t r = 0; r < rows;) {
        const int64_t L = len(r);
        int64_t e = r + 1;
        if (L >= min_len && L <= kBundleMaxLen && inst(r) >= 0)
            while (e < rows && len(e) == L && inst(e) == inst(r) && (!col || shifted(e - 1, e, L)))
                ++e;
        for (int64_t b = r; e - b >= 2; b += kBundleRows)
            out.push_back({(int)b, (int)std::min<int64_t>(kBundleRows, e - b)});
        r = e;
    }
}

// The XCD layout of a schedule's classes into its work-item list.  Heaviest work first so
// the tail of the launch is made of small tiles.  Each class is padded to a multiple of kXCD
// and interleaved: workgroup b runs on XCD b % kXCD, so the item at position kXCD*k + x of
// a class segment is item x*q + k of the class (q = padded length / kXCD): XCD x walks the
// contiguous range [x*q, (x+1)*q).  Whole-workgroup rows are sorted by decreasing length:
// contiguous ranges of a mixed-length list would give the first XCD all the heavy rows.
// Runs of equal length that fill every XCD many times over (e.g. the supply and the demand
// rows of a transportation LP) are range-interleaved; the rest is dealt round-robin, which
// keeps the XCD shares equal.
static void assemble_schedule(Schedule &out) {
    out.items.clear();
    auto append = [&](const std::vector<int4> &src, size_t a, size_t e) {
        if (e <= a) return;
        std::vector<int4> cls(src.begin() + a, src.begin() + e);
        while (cls.size() % kXCD) cls.push_back(make_int4(0, 0, 0, IT_EMPTY));
        const size_t q = cls.size() / kXCD;
        for (size_t k = 0; k < q; ++k)
            for (int x = 0; x < kXCD; ++x) out.items.push_back(cls[x * q + k]);
    };
    const std::vector<int4> &lr = out.cls_long;
    out.items.reserve(out.cls_chunks.size() + out.cls_bundles.size() + lr.size() +
                      out.cls_tiles.size() + 5 * kXCD + lr.size());
    append(out.cls_chunks, 0, out.cls_chunks.size());
    append(out.cls_bundles, 0, out.cls_bundles.size());
    for (size_t a = 0; a < lr.size();) {
        size_t e = a;
        while (e < lr.size() && out.long_len[e] == out.long_len[a]) ++e;
        if (e - a >= (size_t)(16 * kXCD)) append(lr, a, e);
        else out.items.insert(out.items.end(), lr.begin() + a, lr.begin() + e);
        a = e;
    }
    append(out.cls_tiles, 0, out.cls_tiles.size());
    out.n_tiles = (long long)out.cls_tiles.size();
    out.n_rowitems = (long long)lr.size();
    out.n_chunks = (long long)out.cls_chunks.size();
    out.n_bundle_items = (long long)out.cls_bundles.size();
}

void filter_schedule(const Schedule &full, const std::vector<int> &keep, Schedule &out) {
    out = Schedule{};
    out.tile_nnz = full.tile_nnz;
    out.tile_rows = full.tile_rows;
    out.n_chunk_slots = full.n_chunk_slots;
    auto kept = [&](int b) { return b >= 0 && keep[(size_t)b] != 0; };
    for (const int4 &it : full.cls_chunks)
        if (kept(it.z)) out.cls_chunks.push_back(it);
    for (size_t i = 0; i < full.cls_bundles.size(); ++i)
        if (kept(full.bundle_inst[i])) {
            out.cls_bundles.push_back(full.cls_bundles[i]);
            out.bundle_inst.push_back(full.bundle_inst[i]);
        }
    for (size_t i = 0; i < full.cls_long.size(); ++i)
        if (kept(full.cls_long[i].w >> kKindBits)) {
            out.cls_long.push_back(full.cls_long[i]);
            out.long_len.push_back(full.long_len[i]);
        }
    for (const int4 &it : full.cls_tiles)
        if (kept(it.z)) out.cls_tiles.push_back(it);
    for (const int4 &sp : full.splits)
        if (kept(sp.w)) out.splits.push_back(sp);
    assemble_schedule(out);
}

void build_schedule(int64_t rows, const int64_t *rowptr, const ScheduleParams &sp,
                    const int32_t *inst_of_row, const std::vector<Bundle> &bundles,
                    Schedule &out) {
    out.items.clear();
    out.splits.clear();
    out.n_chunk_slots = 0;
    out.tile_nnz = sp.tile_nnz;
    out.tile_rows = sp.tile_rows;
    out.n_bundle_items = 0;
    out.bundle_inst.clear();
    out.long_len.clear();
    std::vector<int4> tiles, longrows, chunks, bitems;
    std::vector<std::pair<int64_t, int64_t>> longlen;  // (len, row) for ordering
    auto inst = [&](int64_t r) { return inst_of_row ? inst_of_row[r] : 0; };
    int64_t r0 = 0, tnnz = 0;
    auto close_tile = [&](int64_t r1) {
        if (r1 > r0) {
            const int nrows = (int)(r1 - r0), cnt = (int)(rowptr[r1] - rowptr[r0]);
            tiles.push_back(make_int4((int)r0, (int)rowptr[r0], inst(r0),
                                      (nrows << 15) | (cnt << kKindBits) | IT_TILE));
        }
        r0 = r1;
        tnnz = 0;
    };
    size_t nb = 0;  // next bundle
    for (int64_t r = 0; r < rows; ++r) {
        const int64_t len = rowptr[r + 1] - rowptr[r];
        if (nb < bundles.size() && bundles[nb].r0 == r) {
            const Bundle bd = bundles[nb++];
            close_tile(r);
            r0 = r + bd.R;
            if (inst(r) >= 0 && len <= kBundleK) {  // one item, epilogue in the item
                bitems.push_back(make_int4((int)r, (int)rowptr[r], inst(r),
                                           (1 << 17) | ((int)(len - 1) << 9) |
                                               ((bd.R - 1) << kKindBits) | IT_BUNDLE));
                out.bundle_inst.push_back(inst(r));
            } else if (inst(r) >= 0) {
                const int C = (int)((len + kBundleK - 1) / kBundleK);
                const int s0 = out.n_chunk_slots;
                for (int c = 0; c < C; ++c) {
                    const int kn = (int)std::min<int64_t>(kBundleK, len - (int64_t)c * kBundleK);
                    bitems.push_back(make_int4((int)r, (int)(rowptr[r] + (int64_t)c * kBundleK * bd.R),
                                               s0 + c, (C << 17) | ((kn - 1) << 9) |
                                                           ((bd.R - 1) << kKindBits) | IT_BUNDLE));
                    out.bundle_inst.push_back(inst(r));
                }
                for (int l = 0; l < bd.R; ++l)
                    out.splits.push_back(make_int4((int)r + l, s0 + l * C, C, inst(r)));
                out.n_chunk_slots += bd.R * C;
            }
            r += bd.R - 1;
            continue;
        }
        if (inst(r) < 0) {  // row of an instance left out of this schedule
            close_tile(r);
            r0 = r + 1;
            continue;
        }
        const bool new_inst = inst_of_row && r > r0 && inst(r) != inst(r0);
        if (len > sp.short_max) {
            close_tile(r);
            r0 = r + 1;
            if (len <= sp.split_len) {
                longlen.push_back({len, r});
            } else {
                const int nch = (int)((len + sp.chunk_nnz - 1) / sp.chunk_nnz);
                out.splits.push_back(make_int4((int)r, out.n_chunk_slots, nch, inst(r)));
                for (int c = 0; c < nch; ++c) {
                    const int64_t p0 = rowptr[r] + (int64_t)c * sp.chunk_nnz;
                    const int64_t p1 = std::min(rowptr[r + 1], p0 + sp.chunk_nnz);
                    chunks.push_back(make_int4((int)p0, (int)p1, inst(r),
                                               ((out.n_chunk_slots + c) << kKindBits) | IT_CHUNK));
                }
                out.n_chunk_slots += nch;
            }
            continue;
        }
        if (new_inst || tnnz + len > sp.tile_nnz || r - r0 >= sp.tile_rows) close_tile(r);
        tnnz += len;
    }
    close_tile(rows);
    std::stable_sort(longlen.begin(), longlen.end(),
                     [](const std::pair<int64_t, int64_t> &a,
                        const std::pair<int64_t, int64_t> &b) { return a.first > b.first; });
    for (auto &lr : longlen) {
        longrows.push_back(make_int4((int)lr.second, (int)rowptr[lr.second],
                                     (int)rowptr[lr.second + 1],
                                     (inst(lr.second) << kKindBits) | IT_ROW));
        out.long_len.push_back(lr.first);
    }
    out.cls_chunks = std::move(chunks);
    out.cls_bundles = std::move(bitems);
    out.cls_long = std::move(longrows);
    out.cls_tiles = std::move(tiles);
    assemble_schedule(out);
}

}  // namespace hprlp
