// Device preprocessing of an LP: the column renumbering, the CSR transpose, the scaling of
// Section 4.1 (Ruiz equilibration, one Pock-Chambolle pass with alpha = 1) and the data
// vectors of the passes.
//
// It produces bit for bit the arrays of the host preprocessing (setup.cpp and api.cpp):
// the same column order (stable by decreasing nonzero count), the same transpose (each
// column lists its rows in increasing order), and the same scaled values.  Ruiz takes
// maxima, which do not depend on order.  The Pock-Chambolle sums run over each row (and
// over each column of the transpose) in storage order, one thread per row, as the host
// does.  Every division and square root in FP64 is correctly rounded on both sides.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hprlp_internal.h"

namespace hprlp {
namespace {

constexpr int kPB = 256;     // threads per block
constexpr int kRadix = 256;  // radix sort: 8 bits per pass

__device__ __forceinline__ int64_t gtid() {
    return (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
}
__device__ __forceinline__ int64_t gstride() { return (int64_t)gridDim.x * blockDim.x; }

int grid_for(int64_t n) {
    const int64_t g = (n + kPB - 1) / kPB;
    return (int)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

int bits_for(uint64_t maxval) {  // bits needed to write every value in [0, maxval]
    int b = 0;
    while (b < 32 && (maxval >> b) != 0) ++b;
    return b;
}

// ------------------------------------------------------------------ elementwise helpers

__global__ void k_iota(uint32_t *v, int64_t n) {
    for (int64_t i = gtid(); i < n; i += gstride()) v[i] = (uint32_t)i;
}

__global__ void k_fill_u32(uint32_t *v, int64_t n, uint32_t x) {
    for (int64_t i = gtid(); i < n; i += gstride()) v[i] = x;
}

__global__ void k_fill_f64(double *v, int64_t n, double x) {
    for (int64_t i = gtid(); i < n; i += gstride()) v[i] = x;
}

__global__ void k_copy_u32(uint32_t *dst, const uint32_t *src, int64_t n) {
    for (int64_t i = gtid(); i < n; i += gstride()) dst[i] = src[i];
}

// counts[key[i]] += 1 (integer atomics: the counts do not depend on the order)
__global__ void k_count(const uint32_t *key, int64_t n, uint32_t *counts) {
    for (int64_t i = gtid(); i < n; i += gstride()) atomicAdd(&counts[key[i]], 1u);
}

// key[j] = total - counts[j]: an ascending stable sort on it orders by decreasing count
__global__ void k_desc_key(const uint32_t *counts, int64_t n, uint32_t total, uint32_t *key) {
    for (int64_t j = gtid(); j < n; j += gstride()) key[j] = total - counts[j];
}

// inv[order[k]] = k; perm_out[k] = order[k] (the renumbering, internal -> caller's column)
__global__ void k_invert(const uint32_t *order, int64_t n, uint32_t *inv, int *perm_out) {
    for (int64_t k = gtid(); k < n; k += gstride()) {
        inv[order[k]] = (uint32_t)k;
        perm_out[k] = (int)order[k];
    }
}

// v[i] = map[v[i]]
__global__ void k_remap(uint32_t *v, int64_t n, const uint32_t *map) {
    for (int64_t i = gtid(); i < n; i += gstride()) v[i] = map[v[i]];
}

// dst[i] = src[idx[i]]
__global__ void k_gather_u32(uint32_t *dst, const uint32_t *src, const uint32_t *idx, int64_t n) {
    for (int64_t i = gtid(); i < n; i += gstride()) dst[i] = src[idx[i]];
}

// dst[i] = src[idx[i]] (idx == nullptr: identity), in FP64 and/or rounded to FP32
__global__ void k_gather_val(double *dst64, float *dst32, const double *src, const uint32_t *idx,
                             int64_t n) {
    for (int64_t i = gtid(); i < n; i += gstride()) {
        const double v = src[idx ? idx[i] : i];
        if (dst64) dst64[i] = v;
        if (dst32) dst32[i] = (float)v;
    }
}

// row[p] = i for every nonzero p of row i (one wavefront per row)
__global__ void k_rowid(const int *rp, int64_t rows, uint32_t *row) {
    const int lane = threadIdx.x & 63;
    const int64_t w0 = gtid() >> 6, nw = gstride() >> 6;
    for (int64_t i = w0; i < rows; i += nw)
        for (int64_t p = rp[i] + lane; p < rp[i + 1]; p += 64) row[p] = (uint32_t)i;
}

// ------------------------------------------------------------------ scans

// Exclusive scan over the block's threads; total = sum of all.  lds: kPB / 64 words.
__device__ uint32_t block_excl_scan(uint32_t v, uint32_t *lds, uint32_t &total) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t x = v;
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t y = __shfl_up(x, o, 64);
        if (lane >= o) x += y;
    }
    if (lane == 63) lds[wave] = x;
    __syncthreads();
    uint32_t before = 0, tot = 0;
    for (int w = 0; w < kPB / 64; ++w) {
        const uint32_t s = lds[w];
        if (w < wave) before += s;
        tot += s;
    }
    __syncthreads();
    total = tot;
    return before + x - v;
}

// Three-step exclusive scan of n unsigned values in place: sums of kScanTile-element
// blocks, their scan (one block), then each block's scan plus its offset.
constexpr int kScanIPT = 16;
constexpr int kScanTile = kPB * kScanIPT;

__global__ __launch_bounds__(kPB) void k_scan_sums(const uint32_t *v, int64_t n, uint32_t *part) {
    __shared__ uint32_t lds[kPB / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    uint32_t s = 0;
    for (int k = 0; k < kScanIPT; ++k) {
        const int64_t i = base + (int64_t)k * kPB + threadIdx.x;
        if (i < n) s += v[i];
    }
    uint32_t tot;
    block_excl_scan(s, lds, tot);
    if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ __launch_bounds__(kPB) void k_scan_top(uint32_t *part, int nb) {
    __shared__ uint32_t lds[kPB / 64];
    uint32_t carry = 0;
    for (int c = 0; c < nb; c += kPB) {
        const int i = c + threadIdx.x;
        const uint32_t v = i < nb ? part[i] : 0u;
        uint32_t tot;
        const uint32_t ex = block_excl_scan(v, lds, tot);
        if (i < nb) part[i] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0) part[nb] = carry;
}

__global__ __launch_bounds__(kPB) void k_scan_apply(const uint32_t *in, int64_t n,
                                                    const uint32_t *part, uint32_t *out) {
    __shared__ uint32_t lds[kPB / 64];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanIPT;
    uint32_t loc[kScanIPT];
    uint32_t s = 0;
    for (int k = 0; k < kScanIPT; ++k) {
        const int64_t i = base + k;
        loc[k] = i < n ? in[i] : 0u;
        s += loc[k];
    }
    uint32_t tot;
    uint32_t run = block_excl_scan(s, lds, tot) + part[blockIdx.x];
    for (int k = 0; k < kScanIPT; ++k) {
        const int64_t i = base + k;
        if (i < n) out[i] = run;
        run += loc[k];
    }
}

int64_t scan_blocks(int64_t n) { return (n + kScanTile - 1) / kScanTile; }

// out[i] = in[0] + ... + in[i-1] (in place allowed); part: scan_blocks(n) + 1 words
hipError_t excl_scan(const uint32_t *in, uint32_t *out, int64_t n, uint32_t *part,
                     hipStream_t st) {
    const int64_t nb = scan_blocks(n);
    if (nb == 0) return hipSuccess;
    k_scan_sums<<<(unsigned)nb, kPB, 0, st>>>(in, n, part);
    k_scan_top<<<1, kPB, 0, st>>>(part, (int)nb);
    k_scan_apply<<<(unsigned)nb, kPB, 0, st>>>(in, n, part, out);
    return hipGetLastError();
}

// ------------------------------------------------------------------ stable radix sort
// LSD radix sort of (key, value) pairs, 8 bits per pass.  Each block owns one tile of
// kSortTile consecutive items: it counts the digits of its tile, the counts are scanned
// digit-major over the tiles, and the block scatters its tile in item order, so equal keys
// keep their input order.

constexpr int kSortIPT = kSortTile / kPB;

__global__ __launch_bounds__(kPB) void k_rs_count(const uint32_t *keys, int64_t n, int shift,
                                                  int ntiles, uint32_t *hist) {
    __shared__ uint32_t cnt[kRadix];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortIPT; ++r) {
        const int64_t i = base + (int64_t)r * kPB + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & (kRadix - 1)], 1u);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// offs: the scanned digit-major counts (first output position of every digit of every tile)
__global__ __launch_bounds__(kPB) void k_rs_scatter(const uint32_t *kin, const uint32_t *vin,
                                                    uint32_t *kout, uint32_t *vout, int64_t n,
                                                    int shift, int ntiles,
                                                    const uint32_t *offs) {
    __shared__ uint32_t run[kRadix];             // next position of every digit
    __shared__ uint32_t wcnt[kPB / 64][kRadix];  // this round: count, then first position,
                                                 // of every digit in every wavefront
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    run[tid] = offs[(int64_t)tid * ntiles + blockIdx.x];
    const int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortIPT; ++r) {
        for (int w = 0; w < kPB / 64; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        const int64_t i = base + (int64_t)r * kPB + tid;
        const bool valid = i < n;
        uint32_t k = 0, v = 0, d = 0;
        if (valid) {
            k = kin[i];
            v = vin[i];
            d = (k >> shift) & (kRadix - 1);
        }
        // lanes of this wavefront holding the same digit
        unsigned long long same = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const bool bit = (d >> b) & 1u;
            const unsigned long long m = __ballot(bit);
            same &= bit ? m : ~m;
        }
        const int rank = __popcll(same & ((1ull << lane) - 1ull));
        if (valid && rank == 0) wcnt[wave][d] = (uint32_t)__popcll(same);
        __syncthreads();
        {   // digit tid: positions of its items in each wavefront, in wavefront order
            uint32_t acc = run[tid];
            for (int w = 0; w < kPB / 64; ++w) {
                const uint32_t c = wcnt[w][tid];
                wcnt[w][tid] = acc;
                acc += c;
            }
            run[tid] = acc;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wcnt[wave][d] + (uint32_t)rank;
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
    }
}

// Sorts (k[0], v[0]) on the low `bits` key bits, using (k[1], v[1]) as the second buffer.
// Returns the index (0 or 1) of the buffers that hold the result.
int radix_sort(uint32_t *k[2], uint32_t *v[2], int64_t n, int bits, uint32_t *hist,
               uint32_t *part, hipStream_t st, hipError_t &err) {
    err = hipSuccess;
    int cur = 0;
    if (n <= 1) return cur;
    const int ntiles = (int)((n + kSortTile - 1) / kSortTile);
    const int64_t hn = (int64_t)kRadix * ntiles;
    for (int shift = 0; shift < bits; shift += 8) {
        k_rs_count<<<ntiles, kPB, 0, st>>>(k[cur], n, shift, ntiles, hist);
        if ((err = hipGetLastError()) != hipSuccess) return cur;
        if ((err = excl_scan(hist, hist, hn, part, st)) != hipSuccess) return cur;
        k_rs_scatter<<<ntiles, kPB, 0, st>>>(k[cur], v[cur], k[1 - cur], v[1 - cur], n, shift,
                                             ntiles, hist);
        if ((err = hipGetLastError()) != hipSuccess) return cur;
        cur = 1 - cur;
    }
    return cur;
}

// ------------------------------------------------------------------ scaling factors

// f[i] = sqrt(max_p |v[p]|) over row i (1 for an empty or zero row): one wavefront per row
__global__ void k_fac_max(const double *v, const int *rp, int64_t rows, double *f) {
    const int lane = threadIdx.x & 63;
    const int64_t w0 = gtid() >> 6, nw = gstride() >> 6;
    for (int64_t i = w0; i < rows; i += nw) {
        double acc = 0.0;
        for (int64_t p = rp[i] + lane; p < rp[i + 1]; p += 64) acc = fmax(acc, fabs(v[p]));
        for (int o = 32; o > 0; o >>= 1) acc = fmax(acc, __shfl_xor(acc, o, 64));
        if (lane == 0) f[i] = acc > 0.0 ? sqrt(acc) : 1.0;
    }
}

// f[i] = sqrt(sum_p |v[p]|) over row i, summed in storage order (one thread per row)
__global__ void k_fac_sum(const double *v, const int *rp, int64_t rows, double *f) {
    for (int64_t i = gtid(); i < rows; i += gstride()) {
        double acc = 0.0;
        for (int64_t p = rp[i]; p < rp[i + 1]; ++p) acc = acc + fabs(v[p]);
        f[i] = acc > 0.0 ? sqrt(acc) : 1.0;
    }
}

// v[p] = v[p] / (rf[row[p]] * cf[col[p]])
__global__ void k_divide(double *v, int64_t n, const uint32_t *row, const int *col,
                         const double *rf, const double *cf) {
    for (int64_t p = gtid(); p < n; p += gstride()) v[p] = v[p] / (rf[row[p]] * cf[col[p]]);
}

// same, with the row and column arrays of the transpose (row of entry q: rowT[q], an int;
// its column: colT[q])
__global__ void k_divide_t(double *v, int64_t n, const int *rowT, const uint32_t *colT,
                           const double *rf, const double *cf) {
    for (int64_t q = gtid(); q < n; q += gstride()) v[q] = v[q] / (rf[rowT[q]] * cf[colT[q]]);
}

__global__ void k_div_vec(double *d, const double *f, int64_t n) {
    for (int64_t i = gtid(); i < n; i += gstride()) d[i] = d[i] / f[i];
}

// ------------------------------------------------------------------ data vectors

__device__ __forceinline__ int inst_of(const int *off, int n_inst, int64_t i) {
    if (!off) return 0;
    int lo = 0, hi = n_inst;  // off[lo] <= i < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}

struct ColVecArgs {
    int64_t n;
    const double *dc, *c, *l, *u;  // c, l, u in the caller's column order
    const int *perm;               // internal column -> caller's column
    const int *col_off;            // nullable (single LP)
    int n_inst;
    const double *cst;             // [n_inst][8]: beta_b, beta_c, ...
    bool mixed, f32;
    double *cd, *ld, *ud, *sc, *co, *cs, *xs, *lo, *uo, *ux;
    float *cd32, *ld32, *ud32, *sc32;
};

__global__ void k_col_vectors(ColVecArgs a) {
    for (int64_t j = gtid(); j < a.n; j += gstride()) {
        const int jc = a.perm[j];
        const double d = a.dc[j], c = a.c[jc], l = a.l[jc], u = a.u[jc];
        const int b = inst_of(a.col_off, a.n_inst, j);
        const double bb = a.cst[(int64_t)b * 8], bc = a.cst[(int64_t)b * 8 + 1];
        double cd, ld, ud;
        if (a.mixed) {  // x' = D_c x~ = x / beta_b
            cd = c / bc;
            ld = l / bb;
            ud = u / bb;
            a.co[j] = bc / (d * d);
            a.cs[j] = 1.0 / d;
            a.xs[j] = 1.0 / d;
            a.ux[j] = bb;
            const double s2 = d * d;
            a.sc[j] = s2;
            if (a.f32) a.sc32[j] = (float)s2;
        } else {        // scaled problem of Section 4.1
            cd = d * c / bc;
            ld = l / d / bb;
            ud = u / d / bb;
            a.co[j] = bc / d;
            a.cs[j] = 1.0;
            a.xs[j] = 1.0;
            a.ux[j] = bb * d;
        }
        a.cd[j] = cd;
        a.ld[j] = ld;
        a.ud[j] = ud;
        a.lo[j] = l;
        a.uo[j] = u;
        if (a.f32) {
            a.cd32[j] = (float)cd;
            a.ld32[j] = (float)ld;
            a.ud32[j] = (float)ud;
        }
    }
}

struct RowVecArgs {
    int64_t m;
    const double *dr, *b;
    const int *row_off;
    int n_inst;
    const double *cst;
    bool mixed, f32;
    double *bd, *sr, *ro, *rs, *ys, *uy;
    float *bd32, *sr32;
};

__global__ void k_row_vectors(RowVecArgs a) {
    for (int64_t i = gtid(); i < a.m; i += gstride()) {
        const double d = a.dr[i], bv = a.b[i];
        const int k = inst_of(a.row_off, a.n_inst, i);
        const double bb = a.cst[(int64_t)k * 8], bc = a.cst[(int64_t)k * 8 + 1];
        double bd;
        if (a.mixed) {  // y' = D_r y~ = y / beta_c
            bd = bv / bb;
            a.ro[i] = bb;
            a.rs[i] = d;
            a.ys[i] = 1.0 / d;
            a.uy[i] = bc;
            const double s2 = d * d;
            a.sr[i] = s2;
            if (a.f32) a.sr32[i] = (float)s2;
        } else {
            bd = d * bv / bb;
            a.ro[i] = bb / d;
            a.rs[i] = 1.0;
            a.ys[i] = 1.0;
            a.uy[i] = bc * d;
        }
        a.bd[i] = bd;
        if (a.f32) a.bd32[i] = (float)bd;
    }
}

#define PREP_CHK(e)                                  \
    do {                                             \
        hipError_t e_ = (e);                         \
        if (e_ != hipSuccess) return e_;             \
    } while (0)
#define PREP_LAUNCH() PREP_CHK(hipGetLastError())

}  // namespace

size_t prep_hist_words(int64_t nnz, int64_t n) {
    const int64_t big = nnz > n ? nnz : n;
    return (size_t)kRadix * (size_t)((big + kSortTile - 1) / kSortTile);
}

size_t prep_part_words(int64_t nnz, int64_t n) {
    const int64_t h = (int64_t)prep_hist_words(nnz, n);
    const int64_t big = h > n + 1 ? h : n + 1;
    return (size_t)scan_blocks(big) + 1;
}

hipError_t prep_matrix(const PrepArgs &a, hipStream_t st) {
    const PrepScratch &s = a.s;
    const int64_t m = a.m, n = a.n, nnz = a.nnz;
    const int gn = grid_for(n), gz = grid_for(nnz), gm = grid_for(m);
    hipError_t err;
    uint32_t *A_ci = reinterpret_cast<uint32_t *>(a.A->ci);
    uint32_t *T_ci = reinterpret_cast<uint32_t *>(a.T->ci);
    uint32_t *T_rp = reinterpret_cast<uint32_t *>(a.T->rp);

    // row of every nonzero (the row ranges of A never change)
    uint32_t *rowid = s.u[4];
    k_rowid<<<grid_for(m * 64), kPB, 0, st>>>(a.A->rp, m, rowid);
    PREP_LAUNCH();

    // column numbering: by decreasing nonzero count, ties in the caller's order
    uint32_t *K[2] = {s.u[0], s.u[1]}, *V[2] = {s.u[2], s.u[3]};
    k_copy_u32<<<gz, kPB, 0, st>>>(K[0], A_ci, nnz);
    PREP_LAUNCH();
    if (a.reorder) {
        k_fill_u32<<<gn, kPB, 0, st>>>(s.cnt, n + 1, 0u);
        k_count<<<gz, kPB, 0, st>>>(K[0], nnz, s.cnt);
        k_desc_key<<<gn, kPB, 0, st>>>(s.cnt, n, (uint32_t)nnz, s.dk[0]);
        k_iota<<<gn, kPB, 0, st>>>(s.dv[0], n);
        PREP_LAUNCH();
        uint32_t *DK[2] = {s.dk[0], s.dk[1]}, *DV[2] = {s.dv[0], s.dv[1]};
        const int r = radix_sort(DK, DV, n, bits_for((uint64_t)nnz), s.hist, s.part, st, err);
        PREP_CHK(err);
        k_invert<<<gn, kPB, 0, st>>>(DV[r], n, s.inv, a.cperm);
        k_remap<<<gz, kPB, 0, st>>>(K[0], nnz, s.inv);  // new column of every nonzero
        PREP_LAUNCH();
    } else {
        k_iota<<<gn, kPB, 0, st>>>(reinterpret_cast<uint32_t *>(a.cperm), n);
        PREP_LAUNCH();
    }

    // row pointers of the transpose: exclusive scan of the column counts
    k_fill_u32<<<gn, kPB, 0, st>>>(s.cnt, n + 1, 0u);
    k_count<<<gz, kPB, 0, st>>>(K[0], nnz, s.cnt);
    PREP_LAUNCH();
    PREP_CHK(excl_scan(s.cnt, T_rp, n + 1, s.part, st));

    // transpose: stable sort of the nonzeros by column -> (column, position in A)
    k_iota<<<gz, kPB, 0, st>>>(V[0], nnz);
    PREP_LAUNCH();
    const int r1 = radix_sort(K, V, nnz, bits_for((uint64_t)(n - 1)), s.hist, s.part, st, err);
    PREP_CHK(err);
    uint32_t *tcol = K[r1], *tpos = V[r1];  // per transposed entry: its column, its raw position
    k_gather_u32<<<gz, kPB, 0, st>>>(T_ci, rowid, tpos, nnz);  // row of every transposed entry
    PREP_LAUNCH();

    // A itself: with renumbered columns every row is re-sorted by its new column indices,
    // which is a second stable sort of the transposed entries, by row
    const uint32_t *apos = nullptr;  // raw position of every nonzero of the final A
    if (a.reorder) {
        uint32_t *K2[2] = {K[1 - r1], s.u[5]}, *V2[2] = {V[1 - r1], A_ci};
        k_copy_u32<<<gz, kPB, 0, st>>>(K2[0], T_ci, nnz);
        k_iota<<<gz, kPB, 0, st>>>(V2[0], nnz);
        PREP_LAUNCH();
        const int r2 = radix_sort(K2, V2, nnz, bits_for((uint64_t)(m - 1)), s.hist, s.part, st, err);
        PREP_CHK(err);
        const uint32_t *qs = V2[r2];  // transposed entry of every slot of A
        uint32_t *ap = K2[0];         // both key buffers are free after the sort
        k_gather_u32<<<gz, kPB, 0, st>>>(ap, tpos, qs, nnz);  // raw position of every slot
        PREP_LAUNCH();
        if (qs == A_ci) {  // the values buffer holding qs is A_ci: move qs out first
            uint32_t *tmp = V2[1 - r2];
            k_copy_u32<<<gz, kPB, 0, st>>>(tmp, qs, nnz);
            PREP_LAUNCH();
            qs = tmp;
        }
        k_gather_u32<<<gz, kPB, 0, st>>>(A_ci, tcol, qs, nnz);
        PREP_LAUNCH();
        apos = ap;
    }

    // values: FP64 -> A~ in place in A.va / T.va; FP32 storage -> the original values in
    // FP32, and FP64 copies in scratch for the scale factors
    double *va = a.mixed ? s.va64 : static_cast<double *>(a.A->va);
    double *vt = a.mixed ? s.vt64 : static_cast<double *>(a.T->va);
    float *va32 = a.mixed ? static_cast<float *>(a.A->va) : nullptr;
    float *vt32 = a.mixed ? static_cast<float *>(a.T->va) : nullptr;
    k_gather_val<<<gz, kPB, 0, st>>>(va, va32, s.vr, apos, nnz);
    k_gather_val<<<gz, kPB, 0, st>>>(vt, vt32, s.vr, tpos, nnz);
    PREP_LAUNCH();

    // column of every transposed entry (tcol) must survive the scaling passes; it lives in
    // K[r1], which the steps above left untouched
    k_fill_f64<<<gm, kPB, 0, st>>>(s.dr, m, 1.0);
    k_fill_f64<<<gn, kPB, 0, st>>>(s.dc, n, 1.0);
    PREP_LAUNCH();
    const int passes = a.ruiz_iters + (a.pock_chambolle ? 1 : 0);
    for (int it = 0; it < passes; ++it) {
        if (it < a.ruiz_iters) {
            k_fac_max<<<grid_for(m * 64), kPB, 0, st>>>(va, a.A->rp, m, s.rf);
            k_fac_max<<<grid_for(n * 64), kPB, 0, st>>>(vt, a.T->rp, n, s.cf);
        } else {
            k_fac_sum<<<gm, kPB, 0, st>>>(va, a.A->rp, m, s.rf);
            k_fac_sum<<<gn, kPB, 0, st>>>(vt, a.T->rp, n, s.cf);
        }
        k_divide<<<gz, kPB, 0, st>>>(va, nnz, rowid, a.A->ci, s.rf, s.cf);
        k_divide_t<<<gz, kPB, 0, st>>>(vt, nnz, a.T->ci, tcol, s.rf, s.cf);
        k_div_vec<<<gm, kPB, 0, st>>>(s.dr, s.rf, m);
        k_div_vec<<<gn, kPB, 0, st>>>(s.dc, s.cf, n);
        PREP_LAUNCH();
    }
    return hipSuccess;
}

hipError_t prep_vectors(const PrepArgs &a, const int *row_off, const int *col_off, int n_inst,
                        const double *cst, const VecSet<double> &d, const VecSet<float> &f,
                        const CheckData &c, double *ux, double *uy, hipStream_t st) {
    const PrepScratch &s = a.s;
    ColVecArgs ca{a.n, s.dc, s.craw, s.lraw, s.uraw, a.cperm, col_off, n_inst, cst,
                  a.mixed, a.f32phase,
                  d.cd, d.ld, d.ud, d.sc, c.co, c.cs, c.xs, c.lo, c.uo, ux,
                  f.cd, f.ld, f.ud, f.sc};
    k_col_vectors<<<grid_for(a.n), kPB, 0, st>>>(ca);
    PREP_LAUNCH();
    RowVecArgs ra{a.m, s.dr, s.braw, row_off, n_inst, cst, a.mixed, a.f32phase,
                  d.bd, d.sr, c.ro, c.rs, c.ys, uy, f.bd, f.sr};
    k_row_vectors<<<grid_for(a.m), kPB, 0, st>>>(ra);
    PREP_LAUNCH();
    return hipSuccess;
}

}  // namespace hprlp
