// Internal declarations shared by the host runtime (api.cpp, setup.cpp) and the HIP kernels
// (kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "hprlp.h"

namespace hprlp {

constexpr int kWG = 256;          // threads per workgroup of the SpMV passes (4 wavefronts)
constexpr int kNQ = 6;            // check quantities per pass (row pass and column pass)

// Work-item kinds of a pass schedule.  One workgroup processes one item; the kind is in
// the low kKindBits bits of the item's w.
enum ItemKind : int { IT_TILE = 0, IT_ROW = 1, IT_CHUNK = 2, IT_EMPTY = 3, IT_BUNDLE = 4 };
constexpr int kKindBits = 3;
constexpr int kKindMask = 7;
// Row bundles: runs of up to 64 consecutive rows of equal length L (L <= kBundleMaxLen; at
// least kBundleMinShifted where each row's columns are its predecessor's plus one, at least
// kBundleMinLen otherwise) whose nonzeros are stored k-major (entry k of the bundle's row l
// at P0 + k R + l, P0 = the first row's offset, R rows), so one lane per row reads the
// stream and, where neighbouring rows hold neighbouring columns, the gathered vector
// coalesced.
constexpr int kBundleRows = 64;
constexpr int kBundleK = 64;       // entries of every row per work item
constexpr int kBundleMinLen = 256;
constexpr int kBundleMinShifted = 16;
constexpr int kBundleMaxLen = 16384;
struct Bundle {
    int r0, R;
};
constexpr int kXCD = 8;           // accelerator complex dies of an MI355X
constexpr int kMaxTileNnz = 2048; // kWG threads x 8 nonzeros (kernels.hip, kEPT)
constexpr int kMaxTileRows = 1024;// kWG threads x 4 rows (kernels.hip, kRPT)

// Schedule of one CSR matrix (host side, then uploaded).  The kind is in the low 3 bits of w.
//   TILE : {r0, P0, inst, nrows << 15 | cnt << 3 | IT_TILE}  rows [r0, r0+nrows), all short,
//          nonzeros [P0, P0+cnt) with cnt <= tile_nnz <= 2048, nrows <= tile_rows <= 1024
//   ROW  : {r, P0, P1, inst << 3 | IT_ROW}     one long row, whole workgroup
//   CHUNK: {p0, p1, inst, slot << 3 | IT_CHUNK} piece of a split row; partial -> split_part[slot]
//   BUNDLE: {r0, p, s, C << 17 | (kn-1) << 9 | (R-1) << 3 | IT_BUNDLE} entries [k0, k0+kn) of
//          the R rows of a bundle (p = P0 + k0 R); row l's partial -> split_part[s + l C],
//          C = the bundle's item count.  C = 1 (L <= kBundleK): the item applies the epilogue
//          itself and s is the instance
//   EMPTY: {0, 0, 0, IT_EMPTY}                 padding so each class starts on an XCD boundary
// splits: {row, slot0, nslots, inst} finished (fixed-order sum + epilogue) by a second kernel.
struct Schedule {
    std::vector<int4> items;
    std::vector<int4> splits;
    int n_chunk_slots = 0;
    int tile_nnz = 0, tile_rows = 0;
    long long n_tiles = 0, n_rowitems = 0, n_chunks = 0, n_bundle_items = 0;
    // the work items of every class before their XCD layout, with what filtering them by
    // instance needs (a batched solve drops the instances that have stopped)
    std::vector<int4> cls_chunks, cls_bundles, cls_long, cls_tiles;
    std::vector<int> bundle_inst;       // instance of every bundle item
    std::vector<int64_t> long_len;      // length of every whole-workgroup row
};

struct ScheduleParams {
    int tile_nnz, tile_rows, short_max, split_len, chunk_nnz;
};

// inst_of_row (nullable): instance of every row; tiles never straddle instances, and rows
// with a negative instance are left out of the schedule (batched solves drop the instances
// that have stopped).  bundles (sorted by r0, inside one instance each): their rows are
// scheduled as BUNDLE items whatever sp says.
void build_schedule(int64_t rows, const int64_t *rowptr, const ScheduleParams &sp,
                    const int32_t *inst_of_row /* nullable */,
                    const std::vector<Bundle> &bundles, Schedule &out);
// The schedule of the instances with keep[b] != 0 from the schedule of all of them: the
// same work items, in the same order, as build_schedule over the kept rows (split slots
// keep their numbers).
void filter_schedule(const Schedule &full, const std::vector<int> &keep, Schedule &out);

// Bundles of the rows of a CSR matrix: every maximal run of >= 2 consecutive rows of one
// instance with equal length in [kBundleMinLen, kBundleMaxLen], cut into pieces of at most
// kBundleRows rows (a last piece of one row is left out).  With col (nullable), a run needs
// instead each row's columns to be its predecessor's plus one (checked at the first, middle
// and last entry), the pattern whose gathers a bundle coalesces, and a length of at least
// kBundleMinShifted.
void find_bundles(int64_t rows, const int64_t *rowptr, const int32_t *col /* nullable */,
                  const int32_t *inst_of_row /* nullable */, std::vector<Bundle> &out);

// A CSR matrix resident in the workspace.
struct DevMat {
    int rows = 0;
    int *rp = nullptr;          // int32[rows+1]
    int *ci = nullptr;          // int32[nnz]
    void *va = nullptr;         // double[nnz] (FP64 mode: scaled A~) or float[nnz] (MIXED: A)
    int4 *items = nullptr;
    int n_items = 0;
    int4 *splits = nullptr;
    int n_split = 0;
    void *split_part = nullptr; // partial sums of split rows (max 16 B per slot)
    int tile_nnz = 0, tile_rows = 0;
    Schedule host;              // kept for stats / re-upload
    // column-ordered tiles: pos[p] = row-order offset inside its tile of the nonzero stored
    // at p (allocated when tile_order allows it); `sorted` says whether the tiles are in that
    // order now.  Whole-workgroup rows and split chunks always keep row order.
    unsigned short *pos = nullptr;
    bool sorted = false;
    // row bundles (fixed at create; their nonzeros are stored k-major from then on)
    std::vector<Bundle> bundles;
    Schedule full;              // batched: the schedule of every instance
};
// Store the nonzeros [P0, P0 + R L) of one bundle k-major, from their row-major copy in
// (tci, tva); values are float (mat_f32) or double.
hipError_t launch_bundle_order(int *ci, void *va, bool mat_f32, const int *tci, const void *tva,
                               long long P0, int R, int L, hipStream_t st);
// Reorder the nonzeros of every tile of M to column order (to_col) or back to row order;
// values are float (mat_f32) or double.
hipError_t launch_tile_order(const DevMat &M, bool mat_f32, bool to_col, hipStream_t st);

// Iterate state and per-iteration data vectors in one precision V.
// Internal coordinates: FP64 mode works on the scaled problem (x~, y~); MIXED works on
// x' = D_c x~ and y' = D_r y~ (= original / beta), with the original FP32-exact A and the
// diagonal scaling folded into the passes (sc = dc^2, sr = dr^2).
template <class V> struct VecSet {
    V *xhat = nullptr, *x0 = nullptr, *cd = nullptr, *ld = nullptr, *ud = nullptr,
      *sc = nullptr;
    // relaxation rho != 2 only: the relaxed point rho x_bar + (1 - rho) x that the Halpern
    // average uses (x_hat then holds 2 x_bar - x, the vector the y-step gathers); nullptr
    // when rho = 2, where the two coincide
    V *xrel = nullptr;
    V *xbar = nullptr, *zint = nullptr, *dx = nullptr;
    V *y = nullptr, *y0 = nullptr, *bd = nullptr, *sr = nullptr;
    V *ybar = nullptr, *dy = nullptr;
};

// MIXED, FP32 phase: the iterate as FP32 displacements from the FP64 anchor w^{r,0} of the
// current outer loop (x0, y0 of d), plus the FP32 data derived from the anchor at every
// restart.  The FP32 pointers alias buffers of the FP32 VecSet (the FP32 copies of c, l, u, b
// and y0 are not needed in this form); d holds the FP64 anchors, data and check outputs.
struct DispSet {
    VecSet<double> d;
    float *dxh = nullptr;    // x_hat - x0 (gathered by the y-step)
    float *dxrel = nullptr;  // relaxed point - x0 (rho != 2 only)
    float *dy = nullptr;     // y - y0 (gathered by the x-step)
    float *q0 = nullptr;     // sc (A^T y0 - c)
    double *q0d = nullptr;   // the same in FP64 (for z_bar in the iterations that keep w_bar)
    float *dl = nullptr, *du = nullptr;  // l - x0, u - x0
    float *sc = nullptr;     // dc^2
    float *r0 = nullptr;     // sr (b - A x0)
    float *ny0 = nullptr;    // -y0
    float *sr = nullptr;     // dr^2
};

// Scalars of one pass launch.
struct IterScalars {
    double sigma;       // sigma_r
    double lam_sigma;   // lambda * sigma_r
    double hx0, hx1;    // x^{r,t} = hx0 * x0 + hx1 * x_hat     (Halpern weights at t)
    double hy0, hy1;    // y^{r,t+1} = hy0 * y0 + hy1 * y_hat   (Halpern weights at t)
    long long m1;       // first inequality row (single LP)
    double rho = 2.0;   // relaxation: w_hat = rho w_bar + (1 - rho) w (2: Peaceman-Rachford)
};

// Per-instance scalars of a batched solve, read by the passes on the device (one set per
// block-diagonal instance; the work items of one instance never mix with another's).
//   t_b = (*kbase + iter_off) - kstart[b] is the inner counter of instance b at this
//   iteration (kbase: iterations completed before the current chunk; iter_off: position of
//   the iteration inside the chunk, fixed when the chunk is captured).
struct BatchArgs {
    const double *sigma = nullptr, *lam = nullptr;
    const long long *kstart = nullptr, *kbase = nullptr;
    const int *m1_end = nullptr;   // absolute index of the instance's first inequality row
    const int *active = nullptr;   // 0 once the instance has stopped
    const double *inv_norm = nullptr;  // power method normalisation per instance
    int iter_off = 0;
    int halpern = 1;
    double rho = 2.0;
};

// Check-pass multipliers (always FP64).
struct CheckData {
    double *ro = nullptr, *rs = nullptr, *ys = nullptr;  // per row
    double *co = nullptr, *cs = nullptr, *xs = nullptr;  // per column
    double *lo = nullptr, *uo = nullptr;                 // original bounds
};

// ---------------------------------------------------------------- kernel launchers
// prec: 0 = FP64 (double A, double vectors, no fold); 1 = MIXED FP32 phase (float A, FP32
// displacements, fold; vecset is a DispSet); 2 = MIXED FP64 phase (float A, double vectors,
// fold).  The check passes take prec 0 or 2 (always FP64 vectors).
// ev_mid (nullable): recorded between the main SpMV kernel and the split-row finisher.
// ba (nullable): batched solve, scalars per instance from device memory instead of s.
hipError_t launch_col_pass(int prec, bool keep, const DevMat &T, const void *vecset,
                           const IterScalars &s, hipStream_t st, hipEvent_t ev_mid = nullptr,
                           const BatchArgs *ba = nullptr);
hipError_t launch_row_pass(int prec, bool keep, const DevMat &A, const void *vecset,
                           const IterScalars &s, hipStream_t st, hipEvent_t ev_mid = nullptr,
                           const BatchArgs *ba = nullptr);
// Check passes: write kNQ partial sums per workgroup slot into parts; then either reduce all
// slots into out[kNQ] (single LP, seg == nullptr) or, per instance b, the slots listed in
// seg->slots[seg->ptr[b] .. seg->ptr[b+1]) into out[b * out_stride + j].
// bd64 / cd64 / sc64: FP64 right-hand side, cost and folded column scaling (dc^2, MIXED only)
struct Segments {
    const int *ptr = nullptr;    // [n_inst + 1]
    const int *slots = nullptr;  // slot indices grouped by instance, in slot order
    int n_inst = 0;
};
hipError_t launch_check_row(int prec, const DevMat &A, const void *vecset, const CheckData &cd,
                            const double *bd64, long long m1, double *parts, double *out,
                            hipStream_t st, const BatchArgs *ba = nullptr,
                            const Segments *seg = nullptr, int out_stride = 0);
hipError_t launch_check_col(int prec, const DevMat &T, const void *vecset, const CheckData &cd,
                            const double *cd64, const double *sc64, double *parts, double *out,
                            hipStream_t st, const BatchArgs *ba = nullptr,
                            const Segments *seg = nullptr, int out_stride = 0);
// power method iteration k (0-based): hist[k] = Rayleigh quotient, inv_norm updated.
// Batched: hist[k * n_inst + b] and inv_norm[b] per instance (segA/segT: slot lists of A, A^T).
hipError_t launch_power_iter(bool mat_f32, bool fold, const DevMat &A, const DevMat &T,
                             double *vg, double *w, const double *sc, const double *sr,
                             double *inv_norm, double *parts_c, double *parts_r, double *hist,
                             int k, hipStream_t st, const BatchArgs *ba = nullptr,
                             const Segments *segA = nullptr, const Segments *segT = nullptr,
                             double *seg_tmp = nullptr);

// Batched decisions (restart criteria, SigmaUpdate, termination) for every instance after a
// chunk of `chunk` iterations; see kernels.hip k_decide for the layout of `dec`.
struct DecideArgs {
    int n_inst, chunk;
    long long max_iter;
    double tol, alpha1, alpha2, alpha3, tol_switch;
    int use_restart, sigma_update;
    const double *res_first;  // [n_inst][2][kNQ] sums of the chunk's first iteration
    const double *res_chk;    // [n_inst][2][kNQ] sums of the chunk's last iteration
    const double *cst;        // [n_inst][8]: beta_b, beta_c, ||b||, ||c||, ||b~||, ||c~||
    double *sigma, *lam, *merit0, *merit_prev;
    long long *kstart, *kbase, *iters_done, *restarts, *nchecks;
    int *active, *status, *restart_flag;
    double *last;             // [n_inst][6]: rel_p, rel_d, rel_gap, pobj, dobj, merit
    double *trace;            // [n_inst][kTraceRows][kTraceCols]
    double *summary;          // [4]: active count, max rel. KKT of active instances, ...
};
constexpr int kTraceRows = 64;
constexpr int kTraceCols = 10;
hipError_t launch_decide(const DecideArgs &d, hipStream_t st);
// w^{r+1,0} = w_bar for the instances flagged by restart_flag (precision V of the set)
hipError_t launch_restart_batched(bool f32, const void *vecset, const int *row_off,
                                  const int *col_off, const int *restart_flag, int n_inst,
                                  hipStream_t st);
hipError_t launch_advance(long long *kbase, int chunk, hipStream_t st);
// MIXED FP32 phase (DispSet): the per-restart FP32 data from the anchor (two FP64 passes);
// the anchor moved to w_bar and the displacements zeroed (one LP, or the instances flagged
// by restart_flag); the switch to FP64 (x_hat, x_rel, y = anchor + displacement).
hipError_t launch_anchor(const DevMat &A, const DevMat &T, const DispSet &v, hipStream_t st);
hipError_t launch_reanchor(const DispSet &v, long long n, long long m, hipStream_t st);
hipError_t launch_reanchor_batched(const DispSet &v, const int *row_off, const int *col_off,
                                   const int *restart_flag, int n_inst, hipStream_t st);
hipError_t launch_disp_promote(const DispSet &v, long long n, long long m, hipStream_t st);
// out[perm[i]] = mul[i] * (a[i] + h * d[i]) (a FP64 anchor, d FP32 displacement)
hipError_t launch_anchor_out(double *out, const double *a, const float *d, double h,
                             const double *mul, const int *perm, long long n, hipStream_t st);
// ---------------------------------------------------------------- device preprocessing
// (prep.hip) The column renumbering, transpose, scaling and data vectors of create, on the
// GPU, with the same results as the host preprocessing.
constexpr int kSortTile = 4096;  // radix sort: items per block

// Scratch of the device preprocessing, carved after the solver's arrays in the workspace.
struct PrepScratch {
    uint32_t *u[6] = {};                       // [nnz] each: sort buffers and index maps
    double *vr = nullptr;                      // [nnz] A's values as given (caller's order)
    double *va64 = nullptr, *vt64 = nullptr;   // [nnz] FP32 storage of A: FP64 scaled copies
    uint32_t *cnt = nullptr;                   // [n + 1] counts, then A^T's row pointers
    uint32_t *dk[2] = {}, *dv[2] = {};         // [n] each: the column-order sort
    uint32_t *inv = nullptr;                   // [n] caller's column -> internal column
    double *rf = nullptr, *cf = nullptr;       // [m], [n] factors of one scaling pass
    double *dr = nullptr, *dc = nullptr;       // [m], [n] products D_r, D_c
    double *braw = nullptr, *craw = nullptr, *lraw = nullptr, *uraw = nullptr;  // as given
    double *cst = nullptr;                     // [n_inst][8] per-instance constants
    uint32_t *hist = nullptr, *part = nullptr; // radix sort digit counts, scan block sums
};

struct PrepArgs {
    int64_t m = 0, n = 0, nnz = 0;
    bool reorder = false, mixed = false, f32phase = false;
    int ruiz_iters = 0;
    bool pock_chambolle = false;
    DevMat *A = nullptr, *T = nullptr;  // in: A.rp, A.ci (caller's columns); out: the rest
    int *cperm = nullptr;               // out: internal column -> caller's column
    PrepScratch s;                      // in: vr, braw, craw, lraw, uraw; out: dr, dc
};

size_t prep_hist_words(int64_t nnz, int64_t n);
size_t prep_part_words(int64_t nnz, int64_t n);
// Column order, A (re-sorted rows), A^T, the scaled values (or FP32 originals) and D_r, D_c.
hipError_t prep_matrix(const PrepArgs &a, hipStream_t st);
// Data vectors in the pass coordinates from D_r, D_c and the per-instance constants cst
// (row_off / col_off: instance offsets on the device, nullptr for one LP).
hipError_t prep_vectors(const PrepArgs &a, const int *row_off, const int *col_off, int n_inst,
                        const double *cst, const VecSet<double> &d, const VecSet<float> &f,
                        const CheckData &c, double *ux, double *uy, hipStream_t st);

// ---------------------------------------------------------------- T1 = 0 (t1zero.hip)
// Section 3.2, item 1: LPs without inequality rows, y-step solved exactly through the
// dense inverse G of A~A~^T (at most kT1MaxRows rows).
constexpr int kT1MaxRows = 65536;  // G takes 8 mp^2 bytes (34 GB at this bound)
size_t t1_parts_len();
// rows of the padded dense arrays: m rounded up to the 64-wide panels
int t1_padded_rows(int m);
// G r from G's lower triangle (when G exceeds 1 GiB): t1_partials_len(m) doubles of
// partials (0 otherwise)
bool t1_lower_product(int m);
size_t t1_partials_len(int m);
// G = (A~A~^T)^{-1} in place in F ([mp][mp], mp = t1_padded_rows(m); G's rows have stride
// mp), by a blocked symmetric sweep; U, V: [mp][64] and Sb: [64][64] scratch; diag0 [m]: the
// diagonal of A~A~^T; diagd [mp]: its LDL^T pivots (for the rank check on the host)
hipError_t t1_build_inverse(const DevMat &A, const DevMat &T, int m, double *F, double *U,
                            double *V, double *Sb, double *diag0, double *diagd,
                            hipStream_t st);
// r = b~ - A~ x_hat through the pass kernel and A's schedule (kernels.hip)
hipError_t launch_t1_resid(const DevMat &A, const double *xhat, const double *bd, double *r,
                           hipStream_t st);
// y-step: r = b~ - A~ x_hat, then y_bar = y + (G r) / sigma and the y update of Algorithm 2;
// P (nullable): the partials of the lower-triangle product
hipError_t t1_row_step(const DevMat &A, const VecSet<double> &v, const IterScalars &s,
                       const double *G, double *r, double *P, int m, bool keep,
                       hipStream_t st);
// *out = ||A~^T (va - vb)||^2 (vb nullable); parts: t1_parts_len() doubles
hipError_t t1_atv_sq(const DevMat &T, int n, const double *va, const double *vb, double *parts,
                     double *out, hipStream_t st);

// vector utilities
hipError_t launch_fill(double *p, long long n, double v, hipStream_t st);
hipError_t launch_fill_f(float *p, long long n, float v, hipStream_t st);
hipError_t launch_copy_d(double *dst, const double *src, long long n, hipStream_t st);
hipError_t launch_copy_f(float *dst, const float *src, long long n, hipStream_t st);
hipError_t launch_f2d(double *dst, const float *src, long long n, hipStream_t st);
// out[perm[i]] = mul[i] * v[i] (mul == nullptr -> scalar smul; perm == nullptr -> identity);
// v in float or double
hipError_t launch_scale_out(double *out, const void *v, bool v_f32, const double *mul,
                            double smul, const int *perm, long long n, hipStream_t st);
// x^{r,t} = hx0 * x0 + hx1 * xhat, scaled by mul/smul, scattered by perm
hipError_t launch_xcur_out(double *out, const void *x0, const void *xhat, bool v_f32,
                           double hx0, double hx1, const double *mul, double smul,
                           const int *perm, long long n, hipStream_t st);

}  // namespace hprlp
