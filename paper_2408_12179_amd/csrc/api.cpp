// C ABI and host driver of the HPR-LP library (Algorithm 2 of the paper).
//
// The iteration runs entirely in the HIP kernels (kernels.hip).  For one LP the host
// launches them and, every check_every iterations (Section 4.1), reads back a dozen reduced
// FP64 scalars to take the termination, restart (Section 3.1) and sigma (Section 3.2,
// Algorithm 3) decisions.  For a batch of LPs packed block-diagonally the same decisions are
// taken per instance on the device, and a whole chunk of check_every iterations (passes,
// check passes, decisions, restart copies) is one hipGraph launch; the host reads back only
// four summary numbers per chunk.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <thread>
#include <mutex>
#include <vector>

#include "hprlp_internal.h"
#include "hprlp_setup.h"

using namespace hprlp;

namespace {

thread_local std::string g_create_error;

enum TraceCol {
    TR_K, TR_T, TR_R, TR_SIGMA, TR_MERIT, TR_MERIT0, TR_MERIT_PREV, TR_REL_P, TR_REL_D,
    TR_REL_GAP, TR_POBJ, TR_DOBJ, TR_DX, TR_DY, TR_ERR_P, TR_ERR_D, TR_RESTART,
    TR_SIGMA_NEW, TR_NCOL
};

double now_ms() {
    return std::chrono::duration<double, std::milli>(
               std::chrono::steady_clock::now().time_since_epoch())
        .count();
}

// Bump allocator over the caller's workspace.
struct Carver {
    char *base;
    size_t cap, used = 0;
    bool dry;  // only count
    void *take(size_t bytes) {
        size_t off = (used + 255) & ~size_t(255);
        used = off + ((bytes + 255) & ~size_t(255));
        if (dry || used > cap) return nullptr;
        return base + off;
    }
    template <class T> T *arr(size_t n) { return static_cast<T *>(take(n * sizeof(T))); }
};

// Candidate values of the schedule autotuner, tried by coordinate descent per matrix: tile
// shape, then the longest row kept in tiles, then the split of very long rows.
constexpr int kTuneTileNnz[] = {1024, 2048};
constexpr int kTuneTileRows[] = {128, 256, 512, 1024};
constexpr int kTuneShortMax[] = {16, 32, 64, 128, 256, 512, 1024, 2048};
constexpr int kTuneSplitLen[] = {2048, 4096, 8192, 16384, 65536};
constexpr int kTuneChunk[] = {2048, 4096, 8192};
constexpr int kTuneMinChunk = 2048, kTuneMinSplit = 2048;
constexpr int64_t kTuneMinNnz = 100000;  // below this a pass is launch-bound: keep the defaults
constexpr int kTuneReps = 10;

// T1 = 0 variant: dense inverse of A~A~^T and its scratch.
struct T1Dev {
    double *G = nullptr;                               // [mp][mp], mp = t1_padded_rows(m)
    double *U = nullptr, *V = nullptr, *S = nullptr;   // [mp][64], [mp][64], [64][64]
    double *r = nullptr, *d0 = nullptr, *dd = nullptr; // [m], [m], [mp]
    double *P = nullptr;    // partials of G r from G's lower triangle (large G only)
    double *parts = nullptr;                           // [t1_parts_len()]
};

// Device arrays of a batched solve (one entry per instance unless noted).
struct BatchDev {
    double *sigma = nullptr, *lam = nullptr, *merit0 = nullptr, *merit_prev = nullptr;
    long long *kstart = nullptr, *kbase = nullptr /*[1]*/, *iters_done = nullptr;
    long long *restarts = nullptr, *nchecks = nullptr;
    int *m1_end = nullptr, *active = nullptr, *status = nullptr, *restart_flag = nullptr;
    int *row_off = nullptr, *col_off = nullptr;   // [n_inst + 1]
    double *inv_norm = nullptr, *cst = nullptr /*[n][8]*/, *last = nullptr /*[n][6]*/;
    double *res_first = nullptr, *res_chk = nullptr;  // [n][2][kNQ]
    double *trace = nullptr;                          // [n][kTraceRows][kTraceCols]
    double *summary = nullptr;                        // [4]
    double *seg_tmp = nullptr;                        // [2n]
    int *segA_ptr = nullptr, *segA_slots = nullptr, *segT_ptr = nullptr, *segT_slots = nullptr;
};

// State of a batched run between hprlp_begin / hprlp_solve and the chunks that follow.
struct BatchRun {
    bool begun = false, done = false;
    double t_start = 0.0, t_power = 0.0;     // host clock (ms) at the start; power method
    int piters = 0;
    long long k = 0, iters_fp32 = 0;         // iterations of the batch; of its FP32 phase
    double prev_active = 0.0;
    int st_all = 0;                          // status of instances still iterating at the end
    std::vector<double> kkt_hist, lam;
    std::vector<std::pair<long long, double>> chunk_end;  // (k, ms since t_start) per chunk
    double prof_ms[2] = {0.0, 0.0};          // profile: summed column / row pass times
    long long prof_n[2] = {0, 0};
};

}  // namespace

struct hprlp_handle {
    hprlp_options opt{};
    int64_t m1 = 0, m2 = 0, m = 0, n = 0, nnz = 0;
    bool mixed = false;     // A stored in FP32 (original values) with the scaling folded
    bool f32phase = false;  // MIXED: starts with FP32 vectors
    hipStream_t st = nullptr;       // stream all library work is ordered on
    hipStream_t user_st = nullptr;  // the caller's stream
    bool own_stream = false;
    bool noalloc = false;                   // created by hprlp_create_noalloc (static scratch)
    hipStream_t cap_st = nullptr;   // single LP: stream the chunk graphs are captured on
    DevMat A, T;
    int *bund_ci = nullptr;         // staging copy of one bundle (create only)
    void *bund_va = nullptr;
    VecSet<double> v64;
    VecSet<float> v32;
    DispSet vdisp;                          // MIXED FP32 phase: displacements (aliases v32)
    CheckData chk;
    double *ux = nullptr, *uy = nullptr;     // unscaling of x and y
    int *cperm = nullptr;                   // column renumbering: internal j -> caller's column
    double *vg = nullptr, *w = nullptr, *hist = nullptr, *inv_norm = nullptr;
    double *partsA = nullptr, *partsT = nullptr;
    double *res = nullptr;                  // [4][kNQ]
    double *outv = nullptr;                 // staging for outputs (n + m + n)
    double *pinned = nullptr;               // host pinned staging
    size_t pinned_len = 0;
    double beta_b = 1, beta_c = 1, bnorm = 0, cnorm = 0, bsnorm = 0, csnorm = 0;
    std::vector<double> dr, dc;
    // batched solve
    bool batched = false;
    int n_inst = 1;
    std::vector<int64_t> row_off;           // instance row offsets (host copy)
    BatchDev bd;
    Segments segA, segT;
    std::vector<double> lam_given;          // per-instance lambda from the caller (or empty)
    hipGraphExec_t graphs[3] = {nullptr, nullptr, nullptr};
    std::vector<hprlp_stats_t> inst_stats;
    BatchRun br;                               // state of the batched run in progress
    bool no_graph_events = false;              // profile: event nodes could not be captured
    std::string graph_event_error;             // why event nodes were refused, if they were
    // schedule parameters of A and A^T (the autotuner may pick different ones per matrix)
    ScheduleParams spA{}, spT{};
    double tuned_ms[2] = {0.0, 0.0};          // autotuner: best row / column pass time
    // schedules over the instances still iterating (rebuilt as instances stop)
    std::vector<int64_t> inst_nnz;            // nonzeros of every instance
    int capA[3] = {0, 0, 0}, capT[3] = {0, 0, 0};  // carved items, splits, chunk slots
    int64_t sched_nnz = 0;                    // nonzeros covered by the current schedules
    bool compacted = false;
    long long n_compactions = 0;
    double t_setup_ms = 0.0;                  // duration of create
    double t_prep_ms = 0.0, t_tune_ms = 0.0;  // create: preprocessing, schedule autotuning
    PrepScratch prep;                         // device preprocessing scratch (create only)
    T1Dev t1;                                 // T1 = 0: inverse of A~A~^T
    // solve state (single LP)
    int prec = 0;
    long long t = 0, k = 0, r = 0;
    double sigma = 1, lambda = 0;
    bool solved = false;
    hprlp_stats_t stats{};
    std::vector<std::array<double, TR_NCOL>> trace;
    std::vector<hipEvent_t> ev_pool;
    std::string err;
};

namespace {

int fail(hprlp_handle *h, int code, const std::string &msg) {
    if (h) h->err = msg;
    else g_create_error = msg;
    return code;
}

#define HIPCHK(h, call)                                                                    \
    do {                                                                                   \
        hipError_t e_ = (call);                                                            \
        if (e_ != hipSuccess)                                                              \
            return fail(h, HPRLP_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)); \
    } while (0)

// Device memory plan; the same function sizes the workspace (dry run) and carves it.
struct Plan {
    int64_t m, n, nnz;
    bool mixed, f32phase;
    bool relax = false;  // rho != 2: a relaxed-x vector per precision set
    int itemsA, itemsT, splitA, splitT, slotsA, slotsT;
    int power_cap;
    int n_inst;
    bool batched;
    bool prep = false;   // scratch of the device preprocessing
    int64_t t1m = 0;     // T1 = 0: rows of the dense inverse of A~A~^T (0: off)
    bool tile_pos = false;  // tiles may be stored in column order: row-order slots per nonzero
    int64_t bundle_tmp = 0; // row bundles possible: entries of the row-major copy of one bundle
};

// Row bundles are possible (every mode but 0).  With T1 = 0 only A's (mode -1): the Gram
// matrix is formed from the row-major A before the bundles are stored, and the check's
// ||A~^T v||^2 reads A~^T row by row.
bool bundles_possible(const hprlp_options &o) { return o.bundle_rows != 0; }

// Column-ordered tiles are possible (forced, or left to the autotuner); never with T1 = 0,
// whose kernels read A row by row.
bool tile_pos_needed(const hprlp_options &o) {
    return !o.t1_zero && (o.tile_order == 1 || (o.tile_order == -1 && o.autotune));
}

void carve(Carver &cv, const Plan &p, hprlp_handle *h) {
    const size_t m = (size_t)p.m, n = (size_t)p.n, nnz = (size_t)p.nnz;
    const size_t vs = p.mixed ? sizeof(float) : sizeof(double);
    DevMat A, T;
    A.rp = cv.arr<int>(m + 1);
    A.ci = cv.arr<int>(nnz);
    A.va = cv.take(nnz * vs);
    T.rp = cv.arr<int>(n + 1);
    T.ci = cv.arr<int>(nnz);
    T.va = cv.take(nnz * vs);
    if (p.tile_pos) {
        A.pos = cv.arr<unsigned short>(nnz);
        T.pos = cv.arr<unsigned short>(nnz);
    }
    A.items = cv.arr<int4>((size_t)std::max(p.itemsA, 1));
    T.items = cv.arr<int4>((size_t)std::max(p.itemsT, 1));
    A.splits = cv.arr<int4>((size_t)std::max(p.splitA, 1));
    T.splits = cv.arr<int4>((size_t)std::max(p.splitT, 1));
    A.split_part = cv.take(16 * (size_t)std::max(p.slotsA, 1));
    T.split_part = cv.take(16 * (size_t)std::max(p.slotsT, 1));
    VecSet<double> d;
    d.xhat = cv.arr<double>(n); d.x0 = cv.arr<double>(n); d.cd = cv.arr<double>(n);
    d.ld = cv.arr<double>(n); d.ud = cv.arr<double>(n);
    d.xbar = cv.arr<double>(n); d.zint = cv.arr<double>(n); d.dx = cv.arr<double>(n);
    d.y = cv.arr<double>(m); d.y0 = cv.arr<double>(m); d.bd = cv.arr<double>(m);
    d.ybar = cv.arr<double>(m); d.dy = cv.arr<double>(m);
    if (p.relax) d.xrel = cv.arr<double>(n);
    VecSet<float> f;
    if (p.mixed) {
        d.sc = cv.arr<double>(n);
        d.sr = cv.arr<double>(m);
    }
    if (p.f32phase) {
        f.xhat = cv.arr<float>(n); f.x0 = cv.arr<float>(n); f.cd = cv.arr<float>(n);
        f.ld = cv.arr<float>(n); f.ud = cv.arr<float>(n); f.sc = cv.arr<float>(n);
        f.xbar = cv.arr<float>(n); f.zint = cv.arr<float>(n); f.dx = cv.arr<float>(n);
        f.y = cv.arr<float>(m); f.y0 = cv.arr<float>(m); f.bd = cv.arr<float>(m);
        f.sr = cv.arr<float>(m); f.ybar = cv.arr<float>(m); f.dy = cv.arr<float>(m);
        if (p.relax) f.xrel = cv.arr<float>(n);
    }
    double *q0d = p.f32phase ? cv.arr<double>(n) : nullptr;
    CheckData c;
    c.ro = cv.arr<double>(m); c.rs = cv.arr<double>(m); c.ys = cv.arr<double>(m);
    c.co = cv.arr<double>(n); c.cs = cv.arr<double>(n); c.xs = cv.arr<double>(n);
    c.lo = cv.arr<double>(n); c.uo = cv.arr<double>(n);
    double *ux = cv.arr<double>(n), *uy = cv.arr<double>(m);
    int *cperm = cv.arr<int>(n);
    double *vg = cv.arr<double>(m), *w = cv.arr<double>(n);
    const size_t ni = (size_t)p.n_inst;
    double *hist = cv.arr<double>((size_t)p.power_cap * ni);
    double *inv_norm = cv.arr<double>(ni);
    double *partsA = cv.arr<double>((size_t)(p.itemsA + p.splitA + 1) * kNQ);
    double *partsT = cv.arr<double>((size_t)(p.itemsT + p.splitT + 1) * kNQ);
    double *res = cv.arr<double>(4 * kNQ);
    double *outv = cv.arr<double>(2 * n + m);
    BatchDev b;
    if (p.batched) {
        b.sigma = cv.arr<double>(ni); b.lam = cv.arr<double>(ni);
        b.merit0 = cv.arr<double>(ni); b.merit_prev = cv.arr<double>(ni);
        b.kstart = cv.arr<long long>(ni); b.kbase = cv.arr<long long>(1);
        b.iters_done = cv.arr<long long>(ni); b.restarts = cv.arr<long long>(ni);
        b.nchecks = cv.arr<long long>(ni);
        b.m1_end = cv.arr<int>(ni); b.active = cv.arr<int>(ni); b.status = cv.arr<int>(ni);
        b.restart_flag = cv.arr<int>(ni);
        b.row_off = cv.arr<int>(ni + 1); b.col_off = cv.arr<int>(ni + 1);
        b.inv_norm = inv_norm;
        b.cst = cv.arr<double>(ni * 8); b.last = cv.arr<double>(ni * 6);
        b.res_first = cv.arr<double>(ni * 2 * kNQ); b.res_chk = cv.arr<double>(ni * 2 * kNQ);
        b.trace = cv.arr<double>(ni * kTraceRows * kTraceCols);
        b.summary = cv.arr<double>(4);
        b.seg_tmp = cv.arr<double>(2 * ni);
        b.segA_ptr = cv.arr<int>(ni + 1);
        b.segA_slots = cv.arr<int>((size_t)(p.itemsA + p.splitA + 1));
        b.segT_ptr = cv.arr<int>(ni + 1);
        b.segT_slots = cv.arr<int>((size_t)(p.itemsT + p.splitT + 1));
    } else {
        // one LP run as captured chunks: sigma, lambda, k_start, k_base in one 32-byte block
        // (one host-to-device copy per chunk), the first inequality row and the active flag
        double *blk = cv.arr<double>(4);
        b.sigma = blk;
        b.lam = blk + 1;
        b.kstart = reinterpret_cast<long long *>(blk + 2);
        b.kbase = reinterpret_cast<long long *>(blk + 3);
        b.m1_end = cv.arr<int>(1);
        b.active = cv.arr<int>(1);
        b.inv_norm = inv_norm;
    }
    T1Dev t1;
    if (p.t1m > 0) {
        const size_t mp = (size_t)t1_padded_rows((int)p.t1m);
        t1.G = cv.arr<double>(mp * mp);
        t1.U = cv.arr<double>(mp * 64); t1.V = cv.arr<double>(mp * 64); t1.S = cv.arr<double>(64 * 64);
        t1.r = cv.arr<double>(m); t1.d0 = cv.arr<double>(m); t1.dd = cv.arr<double>(mp);
        if (t1_partials_len((int)p.t1m) > 0) t1.P = cv.arr<double>(t1_partials_len((int)p.t1m));
        t1.parts = cv.arr<double>(t1_parts_len());
    }
    int *bund_ci = nullptr;
    void *bund_va = nullptr;
    if (p.bundle_tmp > 0) {
        bund_ci = cv.arr<int>((size_t)p.bundle_tmp);
        bund_va = cv.take((size_t)p.bundle_tmp * vs);
    }
    PrepScratch ps;
    if (p.prep) {  // last: nothing of the solve lives after it
        for (auto &b2 : ps.u) b2 = cv.arr<uint32_t>(nnz);
        ps.vr = cv.arr<double>(nnz);
        if (p.mixed) {
            ps.va64 = cv.arr<double>(nnz);
            ps.vt64 = cv.arr<double>(nnz);
        }
        ps.cnt = cv.arr<uint32_t>(n + 1);
        for (int q = 0; q < 2; ++q) {
            ps.dk[q] = cv.arr<uint32_t>(n);
            ps.dv[q] = cv.arr<uint32_t>(n);
        }
        ps.inv = cv.arr<uint32_t>(n);
        ps.rf = cv.arr<double>(m); ps.cf = cv.arr<double>(n);
        ps.dr = cv.arr<double>(m); ps.dc = cv.arr<double>(n);
        ps.braw = cv.arr<double>(m); ps.craw = cv.arr<double>(n);
        ps.lraw = cv.arr<double>(n); ps.uraw = cv.arr<double>(n);
        ps.cst = cv.arr<double>(8 * ni);
        ps.hist = cv.arr<uint32_t>(prep_hist_words(p.nnz, p.n));
        ps.part = cv.arr<uint32_t>(prep_part_words(p.nnz, p.n));
    }
    if (h) {
        h->prep = ps;
        h->t1 = t1;
        h->bund_ci = bund_ci;
        h->bund_va = bund_va;
        h->A.rp = A.rp; h->A.ci = A.ci; h->A.va = A.va; h->A.items = A.items;
        h->A.splits = A.splits; h->A.split_part = A.split_part; h->A.pos = A.pos;
        h->T.rp = T.rp; h->T.ci = T.ci; h->T.va = T.va; h->T.items = T.items;
        h->T.splits = T.splits; h->T.split_part = T.split_part; h->T.pos = T.pos;
        h->v64 = d; h->v32 = f; h->chk = c; h->ux = ux; h->uy = uy; h->vg = vg; h->w = w;
        if (p.f32phase) {
            DispSet &ds = h->vdisp;
            ds.d = d;
            ds.dxh = f.xhat; ds.dxrel = f.xrel; ds.dy = f.y;
            ds.q0 = f.cd; ds.q0d = q0d; ds.dl = f.ld; ds.du = f.ud; ds.sc = f.sc;
            ds.r0 = f.bd; ds.ny0 = f.y0; ds.sr = f.sr;
        }
        h->cperm = cperm;
        h->hist = hist; h->inv_norm = inv_norm; h->partsA = partsA; h->partsT = partsT;
        h->res = res; h->outv = outv;
        h->bd = b;
    }
}

int power_cap(const hprlp_options &o) { return o.power_max_iter + 64; }

size_t plan_bytes(const Plan &p) {
    Carver cv{nullptr, 0, 0, true};
    carve(cv, p, nullptr);
    return cv.used + 256;
}

// Worst-case item counts of a schedule over `rows` rows (see build_schedule): tiles plus
// long rows plus split rows are at most `rows`; chunks at most nnz/chunk + split rows.  A
// batched schedule closes tiles at instance boundaries, which adds at most one tile per
// instance (already inside the 2 * rows bound, as every instance has a row).
Plan bound_plan(int64_t m, int64_t n, int64_t nnz, const hprlp_options &o, int n_inst,
                bool batched) {
    Plan p;
    p.m = m; p.n = n; p.nnz = nnz; p.mixed = o.precision != HPRLP_FP64;
    p.f32phase = o.precision == HPRLP_MIXED;
    p.relax = o.rho != 2.0;
    // with the autotuner on, room for every candidate schedule (smallest chunk and split)
    const int chunk = o.autotune ? std::min(o.chunk_nnz, kTuneMinChunk) : o.chunk_nnz;
    const int split = o.autotune ? std::min(o.split_len, kTuneMinSplit) : o.split_len;
    const int64_t ch = nnz / chunk + 1;
    // padding items: at most kXCD-1 per class segment (chunks, tiles, and each equal-length
    // run of whole-workgroup rows, which has >= 16*kXCD rows): bounded by kXCD + rows/16
    p.itemsA = (int)std::min<int64_t>(2 * m + ch + 3 * kXCD + m / 16, INT32_MAX / 8);
    p.itemsT = (int)std::min<int64_t>(2 * n + ch + 3 * kXCD + n / 16, INT32_MAX / 8);
    p.splitA = (int)std::min<int64_t>(m, nnz / split + 1);
    p.splitT = (int)std::min<int64_t>(n, nnz / split + 1);
    p.slotsA = (int)ch + p.splitA;
    p.slotsT = (int)ch + p.splitT;
    if (bundles_possible(o)) {
        // a bundle has >= 2 rows of >= kBundleMinShifted nonzeros and ceil(L / kBundleK)
        // items: items <= nnz/128 + bundles + padding, bundles <= nnz/(2 kBundleMinShifted).
        // Only bundles of more than kBundleK nonzeros per row use slots (one per row and item)
        // and finishers (one per row): slots <= nnz/64 + such rows <= nnz/64 + nnz/kBundleK
        const int64_t brows = std::min<int64_t>(nnz / kBundleK, std::max(m, n));
        const int64_t bitems = nnz / (2 * kBundleK) + nnz / (2 * kBundleMinShifted) + kXCD;
        p.itemsA = (int)std::min<int64_t>((int64_t)p.itemsA + bitems, INT32_MAX / 8);
        p.itemsT = (int)std::min<int64_t>((int64_t)p.itemsT + bitems, INT32_MAX / 8);
        p.splitA = (int)std::min<int64_t>((int64_t)p.splitA + brows, INT32_MAX / 8);
        p.splitT = (int)std::min<int64_t>((int64_t)p.splitT + brows, INT32_MAX / 8);
        p.slotsA = (int)std::min<int64_t>((int64_t)p.slotsA + nnz / kBundleK + brows, INT32_MAX / 8);
        p.slotsT = (int)std::min<int64_t>((int64_t)p.slotsT + nnz / kBundleK + brows, INT32_MAX / 8);
        p.bundle_tmp = std::min<int64_t>(nnz, (int64_t)kBundleRows * kBundleMaxLen);
    }
    p.power_cap = power_cap(o);
    p.n_inst = n_inst;
    p.batched = batched;
    p.prep = !o.setup_on_host;
    p.t1m = (o.t1_zero && !batched) ? m : 0;
    p.tile_pos = tile_pos_needed(o);
    return p;
}

// Host-to-device copy on the handle's stream; returns once the source may be reused.
template <class T> int upload(hprlp_handle *h, T *dst, const T *src, size_t n) {
    if (n == 0) return HPRLP_OK;
    HIPCHK(h, hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyHostToDevice, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return HPRLP_OK;
}

template <class T> int download(hprlp_handle *h, T *dst, const T *src, size_t n) {
    if (n == 0) return HPRLP_OK;
    HIPCHK(h, hipMemcpyAsync(dst, src, n * sizeof(T), hipMemcpyDeviceToHost, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return HPRLP_OK;
}

hipEvent_t pool_event(hprlp_handle *h, size_t idx) {
    while (h->ev_pool.size() <= idx) {
        hipEvent_t e;
        if (hipEventCreate(&e) != hipSuccess) return nullptr;
        h->ev_pool.push_back(e);
    }
    return h->ev_pool[idx];
}

// Slots of every instance (work items of the main kernel, then split-row finishers), in slot
// order: the check sums of an instance are added in this fixed order.
void build_segments(const Schedule &s, int n_inst, std::vector<int> &ptr,
                    std::vector<int> &slots) {
    std::vector<std::vector<int>> per(n_inst);
    for (size_t p = 0; p < s.items.size(); ++p) {
        const int4 it = s.items[p];
        const int kind = it.w & kKindMask;
        int inst = -1;  // EMPTY items and split BUNDLE items hold no check terms
        if (kind == IT_TILE || kind == IT_CHUNK) inst = it.z;
        else if (kind == IT_ROW) inst = it.w >> kKindBits;
        else if (kind == IT_BUNDLE && (it.w >> 17) == 1) inst = it.z;
        if (inst >= 0) per[inst].push_back((int)p);
    }
    for (size_t q = 0; q < s.splits.size(); ++q)
        per[s.splits[q].w].push_back((int)(s.items.size() + q));
    ptr.assign(n_inst + 1, 0);
    slots.clear();
    for (int b = 0; b < n_inst; ++b) {
        slots.insert(slots.end(), per[b].begin(), per[b].end());
        ptr[b + 1] = (int)slots.size();
    }
}

// Instance structure of a problem (a single LP is one instance).
struct Layout {
    int n_inst;
    std::vector<int64_t> row_off, col_off, m1;
    bool batched;
};

// Host preprocessing path of create: upload A, A^T (int32 row pointers) and the renumbering.
int upload_matrix_host(hprlp_handle *h, const int64_t *rowptr, const int32_t *colidx,
                       const double *val, const std::vector<int64_t> &rpt,
                       const std::vector<int32_t> &cit, const std::vector<int32_t> &pos,
                       const Scaling &sc, const std::vector<int32_t> &order) {
    const int64_t m = h->m, n = h->n, nnz = h->nnz;
    int rc;
    {
        std::vector<int> rp32((size_t)std::max(m, n) + 1);
        for (int64_t i = 0; i <= m; ++i) rp32[i] = (int)rowptr[i];
        if ((rc = upload(h, h->A.rp, rp32.data(), (size_t)m + 1))) return rc;
        for (int64_t j = 0; j <= n; ++j) rp32[j] = (int)rpt[j];
        if ((rc = upload(h, h->T.rp, rp32.data(), (size_t)n + 1))) return rc;
    }
    if ((rc = upload(h, h->cperm, order.data(), (size_t)n))) return rc;
    if ((rc = upload(h, h->A.ci, colidx, (size_t)nnz))) return rc;
    if ((rc = upload(h, h->T.ci, cit.data(), (size_t)nnz))) return rc;
    if (h->mixed) {
        std::vector<float> f((size_t)nnz);
        for (int64_t q = 0; q < nnz; ++q) f[q] = (float)val[q];
        if ((rc = upload(h, (float *)h->A.va, f.data(), (size_t)nnz))) return rc;
        for (int64_t q = 0; q < nnz; ++q) f[q] = (float)val[pos[q]];
        if ((rc = upload(h, (float *)h->T.va, f.data(), (size_t)nnz))) return rc;
    } else {
        if ((rc = upload(h, (double *)h->A.va, sc.val.data(), (size_t)nnz))) return rc;
        std::vector<double> vt((size_t)nnz);
        for (int64_t q = 0; q < nnz; ++q) vt[q] = sc.val[pos[q]];
        if ((rc = upload(h, (double *)h->T.va, vt.data(), (size_t)nnz))) return rc;
    }
    return HPRLP_OK;
}

// Host preprocessing path of create: data vectors in the pass coordinates, check
// multipliers and unscaling; every row and column uses the normalisation factors beta_b,
// beta_c of its own instance.  c, l, u in the internal column order.
int upload_vectors_host(hprlp_handle *h, const double *b, const double *c, const double *l,
                        const double *u, const Scaling &sc, const std::vector<int32_t> &inst_row,
                        const std::vector<int32_t> &inst_col,
                        const std::vector<std::array<double, 8>> &cst) {
    const int64_t m = h->m, n = h->n;
    int rc;
    std::vector<double> cd(n), ld(n), ud(n), bd(m), co(n), csv(n), xs(n), ro(m), rs(m), ys(m),
        ux(n), uy(m), sc2, sr2;
    for (int64_t j = 0; j < n; ++j) {
        const double d = sc.dc[j], bb = cst[inst_col[j]][0], bc = cst[inst_col[j]][1];
        if (h->mixed) {  // x' = D_c x~ = x / beta_b
            cd[j] = c[j] / bc;
            ld[j] = l[j] / bb;
            ud[j] = u[j] / bb;
            co[j] = bc / (d * d);
            csv[j] = 1.0 / d;
            xs[j] = 1.0 / d;
            ux[j] = bb;
        } else {         // scaled problem of Section 4.1
            cd[j] = d * c[j] / bc;
            ld[j] = l[j] / d / bb;
            ud[j] = u[j] / d / bb;
            co[j] = bc / d;
            csv[j] = 1.0;
            xs[j] = 1.0;
            ux[j] = bb * d;
        }
    }
    for (int64_t i = 0; i < m; ++i) {
        const double d = sc.dr[i], bb = cst[inst_row[i]][0], bc = cst[inst_row[i]][1];
        if (h->mixed) {  // y' = D_r y~ = y / beta_c
            bd[i] = b[i] / bb;
            ro[i] = bb;
            rs[i] = d;
            ys[i] = 1.0 / d;
            uy[i] = bc;
        } else {
            bd[i] = d * b[i] / bb;
            ro[i] = bb / d;
            rs[i] = 1.0;
            ys[i] = 1.0;
            uy[i] = bc * d;
        }
    }
    auto up = [&](double *dst, const std::vector<double> &v) {
        return upload(h, dst, v.data(), v.size());
    };
    if ((rc = up(h->v64.cd, cd)) || (rc = up(h->v64.ld, ld)) || (rc = up(h->v64.ud, ud)) ||
        (rc = up(h->v64.bd, bd)) || (rc = up(h->chk.co, co)) || (rc = up(h->chk.cs, csv)) ||
        (rc = up(h->chk.xs, xs)) || (rc = up(h->chk.ro, ro)) || (rc = up(h->chk.rs, rs)) ||
        (rc = up(h->chk.ys, ys)) || (rc = up(h->ux, ux)) || (rc = up(h->uy, uy)))
        return rc;
    if ((rc = upload(h, h->chk.lo, l, (size_t)n)) || (rc = upload(h, h->chk.uo, u, (size_t)n)))
        return rc;
    if (h->mixed) {
        sc2.resize(n);
        sr2.resize(m);
        for (int64_t j = 0; j < n; ++j) sc2[j] = sc.dc[j] * sc.dc[j];
        for (int64_t i = 0; i < m; ++i) sr2[i] = sc.dr[i] * sc.dr[i];
        if ((rc = up(h->v64.sc, sc2)) || (rc = up(h->v64.sr, sr2))) return rc;
    }
    if (h->f32phase) {
        auto upf = [&](float *dst, const std::vector<double> &v) {
            std::vector<float> f(v.size());
            for (size_t i = 0; i < v.size(); ++i) f[i] = (float)v[i];
            return upload(h, dst, f.data(), f.size());
        };
        if ((rc = upf(h->v32.cd, cd)) || (rc = upf(h->v32.ld, ld)) || (rc = upf(h->v32.ud, ud)) ||
            (rc = upf(h->v32.bd, bd)) || (rc = upf(h->v32.sc, sc2)) || (rc = upf(h->v32.sr, sr2)))
            return rc;
    }
    return HPRLP_OK;
}

// Both paths of create: schedules, instance structure and constants, single-LP flags, and
// the pinned staging buffer.
int upload_common(hprlp_handle *h, const Layout &L,
                  const std::vector<std::array<double, 8>> &cst) {
    const hprlp_options &o = h->opt;
    int rc;
    for (DevMat *M : {&h->A, &h->T}) {
        if ((rc = upload(h, M->items, M->host.items.data(), M->host.items.size()))) return rc;
        if ((rc = upload(h, M->splits, M->host.splits.data(), M->host.splits.size())))
            return rc;
    }
    if (!L.batched) {
        const int m1e = (int)L.m1[0], one = 1;
        if ((rc = upload(h, h->bd.m1_end, &m1e, 1)) || (rc = upload(h, h->bd.active, &one, 1)))
            return rc;
    }
    if (L.batched) {
        const int ni = L.n_inst;
        std::vector<int> ro32(ni + 1), co32(ni + 1), m1e(ni);
        std::vector<double> cstf((size_t)ni * 8);
        for (int bi = 0; bi <= ni; ++bi) {
            ro32[bi] = (int)L.row_off[bi];
            co32[bi] = (int)L.col_off[bi];
        }
        for (int bi = 0; bi < ni; ++bi) {
            m1e[bi] = (int)(L.row_off[bi] + L.m1[bi]);
            for (int q = 0; q < 8; ++q) cstf[(size_t)bi * 8 + q] = cst[bi][q];
        }
        std::vector<int> ptr, slots;
        if ((rc = upload(h, h->bd.row_off, ro32.data(), ro32.size())) ||
            (rc = upload(h, h->bd.col_off, co32.data(), co32.size())) ||
            (rc = upload(h, h->bd.m1_end, m1e.data(), m1e.size())) ||
            (rc = upload(h, h->bd.cst, cstf.data(), cstf.size())))
            return rc;
        build_segments(h->A.host, ni, ptr, slots);
        if ((rc = upload(h, h->bd.segA_ptr, ptr.data(), ptr.size())) ||
            (rc = upload(h, h->bd.segA_slots, slots.data(), slots.size())))
            return rc;
        build_segments(h->T.host, ni, ptr, slots);
        if ((rc = upload(h, h->bd.segT_ptr, ptr.data(), ptr.size())) ||
            (rc = upload(h, h->bd.segT_slots, slots.data(), slots.size())))
            return rc;
        h->segA = Segments{h->bd.segA_ptr, h->bd.segA_slots, ni};
        h->segT = Segments{h->bd.segT_ptr, h->bd.segT_slots, ni};
    }
    h->pinned_len = std::max<size_t>(4 * kNQ + 64, (size_t)power_cap(o) * L.n_inst);
    if (h->noalloc) {  // no HIP allocation: pageable host staging (copies then block)
        h->pinned = new (std::nothrow) double[h->pinned_len];
        if (!h->pinned) return fail(h, HPRLP_ENOMEM, "host staging allocation failed");
    } else {
        HIPCHK(h, hipHostMalloc((void **)&h->pinned, h->pinned_len * sizeof(double), 0));
    }
    return HPRLP_OK;
}

// Per instance: beta_b = ||D_r b|| + 1, beta_c = ||D_c c|| + 1 (Section 4.1) and the norms
// the termination test divides by.  dc and c in the internal column order.
std::vector<std::array<double, 8>> instance_constants(const Layout &L, const hprlp_options &o,
                                                      const double *dr, const double *dc,
                                                      const double *b, const double *c) {
    std::vector<std::array<double, 8>> cst(L.n_inst);
    for (int bi = 0; bi < L.n_inst; ++bi) {
        const int64_t r0 = L.row_off[bi], r1 = L.row_off[bi + 1];
        const int64_t c0 = L.col_off[bi], c1 = L.col_off[bi + 1];
        double sb = 0, scc = 0, sbo = 0, sco = 0;
        for (int64_t i = r0; i < r1; ++i) {
            const double v = dr[i] * b[i];
            sb += v * v;
            sbo += b[i] * b[i];
        }
        for (int64_t j = c0; j < c1; ++j) {
            const double v = dc[j] * c[j];
            scc += v * v;
            sco += c[j] * c[j];
        }
        const double bb = o.normalize_bc ? std::sqrt(sb) + 1.0 : 1.0;
        const double bc = o.normalize_bc ? std::sqrt(scc) + 1.0 : 1.0;
        double sbn = 0, scn = 0;  // ||D_r b / beta_b||, ||D_c c / beta_c||
        for (int64_t i = r0; i < r1; ++i) {
            const double v = dr[i] * b[i] / bb;
            sbn += v * v;
        }
        for (int64_t j = c0; j < c1; ++j) {
            const double v = dc[j] * c[j] / bc;
            scn += v * v;
        }
        cst[bi] = {bb, bc, std::sqrt(sbo), std::sqrt(sco), std::sqrt(sbn), std::sqrt(scn), 0.0, 0.0};
    }
    return cst;
}

PrepArgs prep_args(const hprlp_handle *h) {
    PrepArgs a;
    a.m = h->m;
    a.n = h->n;
    a.nnz = h->nnz;
    a.reorder = h->opt.reorder != 0;
    a.mixed = h->mixed;
    a.f32phase = h->f32phase;
    a.ruiz_iters = h->opt.ruiz_iters;
    a.pock_chambolle = h->opt.pock_chambolle != 0;
    a.A = const_cast<DevMat *>(&h->A);
    a.T = const_cast<DevMat *>(&h->T);
    a.cperm = h->cperm;
    a.s = h->prep;
    return a;
}

// Device preprocessing path of create, first part: upload the problem as given, renumber,
// transpose and scale on the GPU, and bring back what the host needs (A^T's row pointers,
// D_r, D_c and the renumbering).  Returns c in the internal column order in c_int.
int prep_on_device(hprlp_handle *h, const int64_t *rowptr, const int32_t *colidx,
                   const double *val, const double *b, const double *c, const double *l,
                   const double *u, std::vector<int64_t> &rpt, std::vector<double> &dr,
                   std::vector<double> &dc, std::vector<double> &c_int) {
    const int64_t m = h->m, n = h->n, nnz = h->nnz;
    const PrepScratch &s = h->prep;
    int rc;
    {
        std::vector<int> rp32((size_t)m + 1);
        for (int64_t i = 0; i <= m; ++i) rp32[i] = (int)rowptr[i];
        if ((rc = upload(h, h->A.rp, rp32.data(), (size_t)m + 1))) return rc;
    }
    if ((rc = upload(h, h->A.ci, colidx, (size_t)nnz)) || (rc = upload(h, s.vr, val, (size_t)nnz)) ||
        (rc = upload(h, s.braw, b, (size_t)m)) || (rc = upload(h, s.craw, c, (size_t)n)) ||
        (rc = upload(h, s.lraw, l, (size_t)n)) || (rc = upload(h, s.uraw, u, (size_t)n)))
        return rc;
    PrepArgs a = prep_args(h);
    HIPCHK(h, prep_matrix(a, h->st));
    std::vector<int> t32((size_t)n + 1), order((size_t)n);
    dr.resize((size_t)m);
    dc.resize((size_t)n);
    if ((rc = download(h, t32.data(), h->T.rp, (size_t)n + 1)) ||
        (rc = download(h, order.data(), h->cperm, (size_t)n)) ||
        (rc = download(h, dr.data(), s.dr, (size_t)m)) ||
        (rc = download(h, dc.data(), s.dc, (size_t)n)))
        return rc;
    rpt.resize((size_t)n + 1);
    for (int64_t j = 0; j <= n; ++j) rpt[j] = t32[j];
    c_int.resize((size_t)n);
    for (int64_t j = 0; j < n; ++j) c_int[j] = c[order[j]];
    h->dr = dr;
    h->dc.assign((size_t)n, 1.0);
    for (int64_t j = 0; j < n; ++j) h->dc[order[j]] = dc[j];  // caller's column order
    return HPRLP_OK;
}

// Block structure of a batched problem (host only, after validate_problem).
int validate_layout(const Layout &L, int64_t m, int64_t n, const int64_t *rowptr,
                    const int32_t *colidx, std::string &err) {
    const int ni = L.n_inst;
    if (L.row_off[0] != 0 || L.col_off[0] != 0 || L.row_off[ni] != m || L.col_off[ni] != n) {
        err = "instance offsets must start at 0 and end at m and n";
        return HPRLP_EDIM;
    }
    for (int b = 0; b < ni; ++b) {
        if (L.row_off[b + 1] <= L.row_off[b] || L.col_off[b + 1] <= L.col_off[b]) {
            err = "instance " + std::to_string(b) + " has no rows or no columns";
            return HPRLP_EDIM;
        }
        if (L.m1[b] < 0 || L.m1[b] > L.row_off[b + 1] - L.row_off[b]) {
            err = "instance " + std::to_string(b) + ": m1 out of range";
            return HPRLP_EDIM;
        }
        if (rowptr[L.row_off[b + 1]] == rowptr[L.row_off[b]]) {
            err = "instance " + std::to_string(b) + " has an empty matrix";
            return HPRLP_EDIM;
        }
        for (int64_t i = L.row_off[b]; i < L.row_off[b + 1]; ++i)
            for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
                if (colidx[p] < L.col_off[b] || colidx[p] >= L.col_off[b + 1]) {
                    err = "row " + std::to_string(i) + " reaches outside its instance's columns";
                    return HPRLP_EDIM;
                }
    }
    return HPRLP_OK;
}

int tune_schedules(hprlp_handle *h, const int64_t *rpA, const int64_t *rpT,
                   const int32_t *inst_row, const int32_t *inst_col);
int set_tile_order(hprlp_handle *h, bool row, bool col, bool to_col);

// Row bundles of A and A^T for options o (fixed at create): found on the caller's arrays.
// Rows keep their order; A^T's rows are the columns, after the renumbering by decreasing
// count when o.reorder (so its row lengths are the column counts, sorted).  rpT (nullable)
// receives those row pointers when A^T is searched.
void detect_bundles(const hprlp_options &o, int64_t m, int64_t n, const int64_t *rowptr,
                    const int32_t *colidx, const int32_t *irow, const int32_t *icol,
                    std::vector<Bundle> &bA, std::vector<Bundle> &bT,
                    std::vector<int64_t> *rpT_out) {
    bA.clear();
    bT.clear();
    if (!bundles_possible(o)) return;
    find_bundles(m, rowptr, o.bundle_rows == 1 ? nullptr : colidx, irow, bA);
    if (o.bundle_rows == 1) {
        const int64_t nnz = rowptr[m];
        std::vector<int64_t> deg((size_t)n, 0), rpT((size_t)n + 1, 0);
        for (int64_t p = 0; p < nnz; ++p) deg[colidx[p]]++;
        if (o.reorder) std::stable_sort(deg.begin(), deg.end(), std::greater<int64_t>());
        for (int64_t j = 0; j < n; ++j) rpT[j + 1] = rpT[j] + deg[j];
        find_bundles(n, rpT.data(), nullptr, icol, bT);
        if (rpT_out) *rpT_out = std::move(rpT);
    }
}

// Store every bundle's nonzeros k-major (once, after the preprocessing): each bundle is
// copied to the staging buffer, then written back in its new order.
int store_bundles(hprlp_handle *h, const int64_t *rpA, const int64_t *rpT) {
    for (int w = 0; w < 2; ++w) {
        DevMat &M = w ? h->T : h->A;
        const int64_t *rp = w ? rpT : rpA;
        const size_t vs = h->mixed ? sizeof(float) : sizeof(double);
        for (const Bundle &b : M.bundles) {
            const long long P0 = rp[b.r0];
            const int L = (int)(rp[b.r0 + 1] - rp[b.r0]);
            if (rp[b.r0 + b.R] - P0 != (int64_t)b.R * L || L < kBundleMinShifted || L > kBundleMaxLen)
                return fail(h, HPRLP_EHIP, "row bundle " + std::to_string(b.r0) +
                                               ": rows of unequal length (internal error)");
            const size_t cnt = (size_t)b.R * (size_t)L;
            HIPCHK(h, hipMemcpyAsync(h->bund_ci, M.ci + P0, cnt * sizeof(int),
                                     hipMemcpyDeviceToDevice, h->st));
            HIPCHK(h, hipMemcpyAsync(h->bund_va, static_cast<char *>(M.va) + P0 * vs, cnt * vs,
                                     hipMemcpyDeviceToDevice, h->st));
            HIPCHK(h, launch_bundle_order(M.ci, M.va, h->mixed, h->bund_ci, h->bund_va, P0, b.R,
                                          L, h->st));
        }
    }
    HIPCHK(h, hipStreamSynchronize(h->st));
    return HPRLP_OK;
}

// Where the T1 = 0 variant applies: one LP, equality rows only, FP64, a dense inverse of
// A~A~^T of at most kT1MaxRows rows.
int t1_check(const hprlp_options &o, bool batched, int64_t m, int64_t m2, std::string &err) {
    if (!o.t1_zero) return HPRLP_OK;
    if (batched) { err = "t1_zero applies to single LPs"; return HPRLP_EINVAL; }
    if (m2 != 0) { err = "t1_zero needs an LP without inequality rows (m2 = 0)"; return HPRLP_EINVAL; }
    if (o.precision != HPRLP_FP64) { err = "t1_zero runs in FP64 only"; return HPRLP_EINVAL; }
    if (m > kT1MaxRows) {
        err = "t1_zero: at most " + std::to_string(kT1MaxRows) + " rows (dense inverse of A A^T)";
        return HPRLP_EDIM;
    }
    return HPRLP_OK;
}

// Build G = (A~A~^T)^{-1} and reject A without full row rank (a pivot of LDL^T at most
// 1e-10 times its diagonal entry of A~A~^T).
int t1_setup(hprlp_handle *h) {
    const int m = (int)h->m;
    HIPCHK(h, t1_build_inverse(h->A, h->T, m, h->t1.G, h->t1.U, h->t1.V, h->t1.S, h->t1.d0,
                               h->t1.dd, h->st));
    std::vector<double> d0((size_t)m), dd((size_t)m);
    int rc;
    if ((rc = download(h, d0.data(), h->t1.d0, (size_t)m)) ||
        (rc = download(h, dd.data(), h->t1.dd, (size_t)m)))
        return rc;
    for (int k = 0; k < m; ++k)
        if (!(dd[k] > 1e-10 * d0[k]) || !std::isfinite(dd[k]))
            return fail(h, HPRLP_EINVAL, "t1_zero needs A of full row rank: A A^T is singular "
                                         "(LDL^T pivot " + std::to_string(k) + ")");
    return HPRLP_OK;
}

// Shared body of hprlp_create and hprlp_create_batched.
int create_impl(hprlp_handle **out, const Layout &L, const int64_t *rowptr,
                const int32_t *colidx, const double *val, const double *b, const double *c,
                const double *l, const double *u, const double *lambda_inst,
                const hprlp_options *opt, void *d_workspace, size_t ws_bytes, void *stream,
                bool noalloc = false) {
    if (!out) return fail(nullptr, HPRLP_EINVAL, "out is null");
    *out = nullptr;
    const double t_create = now_ms();
    hprlp_options o;
    if (opt) o = *opt;
    else hprlp_default_options(&o);
    resolve_options(o);
    if (L.batched) o.reorder = 0;  // instances keep their own contiguous column blocks
    std::string err;
    int rc = validate_options(o, err);
    if (rc) return fail(nullptr, rc, err);
    if (L.batched && o.check_every < 2)
        return fail(nullptr, HPRLP_EINVAL, "batched solves need check_every >= 2");
    const int64_t m = L.row_off[L.n_inst], n = L.col_off[L.n_inst];
    int64_t m1tot = 0;
    for (int bi = 0; bi < L.n_inst; ++bi) m1tot += L.m1[bi];
    if ((rc = t1_check(o, L.batched, m, m - m1tot, err))) return fail(nullptr, rc, err);
    if (o.t1_zero) o.graph = 0;  // the chunk graphs capture the lambda-variant passes
    rc = validate_problem(L.batched ? m : L.m1[0], L.batched ? 0 : m - L.m1[0], n, rowptr,
                          colidx, val, b, c, l, u, o, err);
    if (rc) return fail(nullptr, rc, err);
    if (L.batched && (rc = validate_layout(L, m, n, rowptr, colidx, err)))
        return fail(nullptr, rc, err);
    if (lambda_inst)
        for (int bi = 0; bi < L.n_inst; ++bi)
            if (!(lambda_inst[bi] > 0.0) || !std::isfinite(lambda_inst[bi]))
                return fail(nullptr, HPRLP_EINVAL, "lambda values must be positive and finite");
    if (!d_workspace || (reinterpret_cast<uintptr_t>(d_workspace) & 255))
        return fail(nullptr, HPRLP_EINVAL, "workspace must be a non-null 256-byte aligned device pointer");

    const int64_t nnz = rowptr[m];
    hprlp_handle *h = new (std::nothrow) hprlp_handle();
    if (!h) return fail(nullptr, HPRLP_ENOMEM, "handle allocation failed");
    h->opt = o; h->m = m; h->n = n; h->nnz = nnz;
    h->m1 = L.batched ? m1tot : L.m1[0];
    h->m2 = m - h->m1;
    h->mixed = o.precision != HPRLP_FP64;
    h->f32phase = o.precision == HPRLP_MIXED;
    h->batched = L.batched;
    h->n_inst = L.n_inst;
    h->row_off = L.row_off;
    h->user_st = static_cast<hipStream_t>(stream);
    h->st = h->user_st;
    h->noalloc = noalloc;
    if (lambda_inst) h->lam_given.assign(lambda_inst, lambda_inst + L.n_inst);

    // instance of every row and column
    std::vector<int32_t> inst_row((size_t)m), inst_col((size_t)n);
    for (int bi = 0; bi < L.n_inst; ++bi) {
        for (int64_t i = L.row_off[bi]; i < L.row_off[bi + 1]; ++i) inst_row[i] = bi;
        for (int64_t j = L.col_off[bi]; j < L.col_off[bi + 1]; ++j) inst_col[j] = bi;
    }
    const ScheduleParams spar{o.tile_nnz, o.tile_rows, o.short_max, o.split_len, o.chunk_nnz};
    h->spA = h->spT = spar;
    const int32_t *irow = L.batched ? inst_row.data() : nullptr;
    const int32_t *icol = L.batched ? inst_col.data() : nullptr;
    auto build_schedules = [&](const int64_t *rpT) {
        build_schedule(m, rowptr, spar, irow, h->A.bundles, h->A.host);
        build_schedule(n, rpT, spar, icol, h->T.bundles, h->T.host);
        for (DevMat *M : {&h->A, &h->T}) {
            M->n_items = (int)M->host.items.size();
            M->n_split = (int)M->host.splits.size();
            M->tile_nnz = M->host.tile_nnz;
            M->tile_rows = M->host.tile_rows;
        }
    };
    // carve the workspace (sizes: the schedules already built, or the bound over every
    // autotuner candidate) and set up the stream; false + h deleted on failure
    auto carve_all = [&](Plan need) -> int {
        if (plan_bytes(need) > ws_bytes) {
            delete h;
            return fail(nullptr, HPRLP_EINVAL, "workspace too small: need " +
                                                   std::to_string(plan_bytes(need)) + " bytes");
        }
        Carver cv{static_cast<char *>(d_workspace), ws_bytes, 0, false};
        carve(cv, need, h);
        h->A.rows = (int)m;
        h->T.rows = (int)n;
        h->capA[0] = need.itemsA; h->capA[1] = need.splitA; h->capA[2] = need.slotsA;
        h->capT[0] = need.itemsT; h->capT[1] = need.splitT; h->capT[2] = need.slotsT;
        h->sched_nnz = nnz;
        if (L.batched) {
            // batched work is ordered on a stream of the library's own (stream capture needs
            // a stream other than the legacy default one); each entry point first waits for
            // the caller's stream
            if (h->user_st && hipStreamSynchronize(h->user_st) != hipSuccess) {
                delete h;
                return fail(nullptr, HPRLP_EHIP, "caller stream synchronisation failed");
            }
            if (hipStreamCreateWithFlags(&h->st, hipStreamNonBlocking) != hipSuccess) {
                delete h;
                return fail(nullptr, HPRLP_EHIP, "hipStreamCreateWithFlags failed");
            }
            h->own_stream = true;
        }
        return HPRLP_OK;
    };
    // Row bundles, fixed for the handle's lifetime
    detect_bundles(o, m, n, rowptr, colidx, irow, icol, h->A.bundles, h->T.bundles, nullptr);
    Plan need = bound_plan(m, n, nnz, o, L.n_inst, L.batched);
    std::vector<int64_t> rpt;
    std::vector<std::array<double, 8>> cst;
    const double t_prep = now_ms();

    if (o.setup_on_host) {
        // ---- host preprocessing
        // Column renumbering by decreasing nonzero count (single LP): the most gathered
        // entries of x_hat then share cache lines.  It permutes the variables only; every
        // output is scattered back to the caller's order.
        std::vector<int32_t> order((size_t)n), colr;
        std::vector<double> valr, cr, lr, ur;
        for (int64_t j = 0; j < n; ++j) order[j] = (int32_t)j;
        if (o.reorder) {
            std::vector<int64_t> deg((size_t)n, 0);
            for (int64_t p = 0; p < nnz; ++p) deg[colidx[p]]++;
            std::stable_sort(order.begin(), order.end(),
                             [&](int32_t a, int32_t b2) { return deg[a] > deg[b2]; });
            std::vector<int32_t> inv((size_t)n);
            for (int64_t j = 0; j < n; ++j) inv[order[j]] = (int32_t)j;
            colr.resize((size_t)nnz);
            valr.resize((size_t)nnz);
            std::vector<std::pair<int32_t, double>> rowbuf;
            for (int64_t i = 0; i < m; ++i) {
                rowbuf.clear();
                for (int64_t p = rowptr[i]; p < rowptr[i + 1]; ++p)
                    rowbuf.push_back({inv[colidx[p]], val[p]});
                std::sort(rowbuf.begin(), rowbuf.end(),
                          [](const std::pair<int32_t, double> &a,
                             const std::pair<int32_t, double> &b2) { return a.first < b2.first; });
                for (size_t q = 0; q < rowbuf.size(); ++q) {
                    colr[rowptr[i] + q] = rowbuf[q].first;
                    valr[rowptr[i] + q] = rowbuf[q].second;
                }
            }
            cr.resize((size_t)n); lr.resize((size_t)n); ur.resize((size_t)n);
            for (int64_t j = 0; j < n; ++j) {
                cr[j] = c[order[j]];
                lr[j] = l[order[j]];
                ur[j] = u[order[j]];
            }
            colidx = colr.data();
            val = valr.data();
            c = cr.data();
            l = lr.data();
            u = ur.data();
        }
        std::vector<int32_t> cit, pos;
        transpose(m, n, rowptr, colidx, rpt, cit, pos);
        Scaling sc;
        precondition(m, n, rowptr, colidx, rpt, pos, val, o, sc);
        h->dr = sc.dr;
        h->dc.assign((size_t)n, 1.0);
        for (int64_t j = 0; j < n; ++j) h->dc[order[j]] = sc.dc[j];  // caller's column order
        cst = instance_constants(L, o, sc.dr.data(), sc.dc.data(), b, c);
        build_schedules(rpt.data());
        if (!o.autotune) {
            need.itemsA = (int)h->A.host.items.size();
            need.itemsT = (int)h->T.host.items.size();
            need.splitA = (int)h->A.host.splits.size();
            need.splitT = (int)h->T.host.splits.size();
            need.slotsA = h->A.host.n_chunk_slots;
            need.slotsT = h->T.host.n_chunk_slots;
        }
        if ((rc = carve_all(need))) return rc;
        rc = upload_matrix_host(h, rowptr, colidx, val, rpt, cit, pos, sc, order);
        if (!rc) rc = upload_vectors_host(h, b, c, l, u, sc, inst_row, inst_col, cst);
        if (!rc) rc = upload_common(h, L, cst);
    } else {
        // ---- device preprocessing: the same arrays, computed in the workspace
        if ((rc = carve_all(need))) return rc;
        std::vector<double> dr, dc, c_int;
        rc = prep_on_device(h, rowptr, colidx, val, b, c, l, u, rpt, dr, dc, c_int);
        if (!rc) {
            cst = instance_constants(L, o, dr.data(), dc.data(), b, c_int.data());
            build_schedules(rpt.data());
            rc = upload_common(h, L, cst);
        }
        if (!rc && !L.batched) {
            std::vector<double> c0(cst[0].begin(), cst[0].end());
            rc = upload(h, h->prep.cst, c0.data(), c0.size());
        }
        if (!rc) {
            const PrepArgs a = prep_args(h);
            const double *dcst = L.batched ? h->bd.cst : h->prep.cst;
            hipError_t e = prep_vectors(a, L.batched ? h->bd.row_off : nullptr,
                                        L.batched ? h->bd.col_off : nullptr, L.n_inst, dcst,
                                        h->v64, h->v32, h->chk, h->ux, h->uy, h->st);
            if (e == hipSuccess) e = hipStreamSynchronize(h->st);
            if (e != hipSuccess)
                rc = fail(h, HPRLP_EHIP, std::string("device preprocessing: ") + hipGetErrorString(e));
        }
    }
    if (!rc) {  // single LP: the normalisation and the norms of the termination test
        h->beta_b = cst[0][0];
        h->beta_c = cst[0][1];
        h->bnorm = cst[0][2];
        h->cnorm = cst[0][3];
        h->bsnorm = cst[0][4];
        h->csnorm = cst[0][5];
    }
    if (!rc && o.t1_zero) rc = t1_setup(h);
    if (!rc) rc = store_bundles(h, rowptr, rpt.data());
    h->t_prep_ms = now_ms() - t_prep;
    const double t_tune = now_ms();
    if (!rc && o.autotune && nnz >= kTuneMinNnz)
        rc = tune_schedules(h, rowptr, rpt.data(), irow, icol);
    if (!rc && o.tile_order == 1 && h->A.pos) rc = set_tile_order(h, true, true, true);
    h->t_tune_ms = now_ms() - t_tune;
    if (rc) {
        g_create_error = h->err;
        hprlp_destroy(h);
        return rc;
    }
    if (L.batched) {  // kept to filter the schedules to the instances still iterating
        h->A.full = h->A.host;
        h->T.full = h->T.host;
        h->inst_nnz.assign(L.n_inst, 0);
        for (int bi = 0; bi < L.n_inst; ++bi)
            h->inst_nnz[bi] = rowptr[L.row_off[bi + 1]] - rowptr[L.row_off[bi]];
    }
    h->t_setup_ms = now_ms() - t_create;
    *out = h;
    return HPRLP_OK;
}

int workspace_impl(int32_t n_inst, int64_t m, int64_t n, int64_t nnz, const hprlp_options *opt,
                   size_t *bytes, bool batched);

}  // namespace

// ---------------------------------------------------------------------------- static scratch
//
// The workspace of hprlp_create_noalloc: a file-scope device array, one copy per GPU (part
// of the code object the runtime loads on each device the library runs on, held until the
// process ends).  Host code never passes the array's name to a kernel or a copy (on the host
// it is only a stand-in symbol): the device address comes from hipGetSymbolAddress, taken
// once per device with that device current, and is the only pointer used afterwards.
constexpr size_t kScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kMaxDevices] = {};
const hprlp_handle *g_scratch_owner[kMaxDevices] = {};  // live noalloc handle per device
int g_scratch_dev_of(const hprlp_handle *h) {
    for (int d = 0; d < kMaxDevices; ++d)
        if (g_scratch_owner[d] == h) return d;
    return -1;
}

void release_scratch(const hprlp_handle *h) {
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    const int d = g_scratch_dev_of(h);
    if (d >= 0) g_scratch_owner[d] = nullptr;
}

// ============================================================================ C ABI

extern "C" void hprlp_default_options(hprlp_options *o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->tol = 1e-8;
    o->check_every = 150;
    o->max_iter = 10000000;
    o->time_limit = 0;
    o->alpha1 = 0.2;
    o->alpha2 = 0.6;
    o->alpha3 = 0.2;
    o->sigma0 = 1.0;
    o->ruiz_iters = 10;
    o->pock_chambolle = 1;
    o->normalize_bc = 1;
    o->power_max_iter = 5000;
    o->power_tol = 1e-10;
    o->lambda_override = 0;
    o->use_halpern = 1;
    o->use_restart = 1;
    o->sigma_update = 1;
    o->precision = HPRLP_FP64;
    o->tol_switch = 1e-5;
    o->stall_checks = 0;
    o->reorder = 1;
    o->profile = 0;
    o->verbose = 0;
    o->autotune = 0;
    o->stall_ratio = 0.5;
    o->graph = 1;
    o->rho = 2.0;
    o->tile_order = 0;
    o->bundle_rows = -1;
    resolve_options(*o);
}

namespace {
int workspace_impl(int32_t n_inst, int64_t m, int64_t n, int64_t nnz, const hprlp_options *opt,
                   size_t *bytes, bool batched) {
    hprlp_options o;
    if (opt) o = *opt;
    else hprlp_default_options(&o);
    resolve_options(o);
    if (!bytes) return fail(nullptr, HPRLP_EINVAL, "bytes is null");
    if (n_inst < 1 || m < 1 || n < 1 || nnz < 1 || nnz >= (1LL << 31) || m >= (1LL << 31) ||
        n >= (1LL << 31) || n_inst > m || n_inst > n)
        return fail(nullptr, HPRLP_EDIM, "bad dimensions");
    std::string err;
    int rc = validate_options(o, err);
    if (rc) return fail(nullptr, rc, err);
    *bytes = plan_bytes(bound_plan(m, n, nnz, o, n_inst, batched));
    return HPRLP_OK;
}
}  // namespace

extern "C" int hprlp_workspace_bytes(int64_t m1, int64_t m2, int64_t n, int64_t nnz,
                                     const hprlp_options *opt, size_t *bytes) {
    if (m1 < 0 || m2 < 0) return fail(nullptr, HPRLP_EDIM, "bad dimensions");
    if (opt) {
        std::string err;
        if (int rc = t1_check(*opt, false, m1 + m2, m2, err)) return fail(nullptr, rc, err);
    }
    return workspace_impl(1, m1 + m2, n, nnz, opt, bytes, false);
}

extern "C" int hprlp_plan_schedule(int64_t m, int64_t n, const int64_t *rowptr,
                                   const int32_t *colidx, const hprlp_options *opt, int matrix,
                                   int64_t *counts) {
    if (m < 1 || n < 1) return fail(nullptr, HPRLP_EDIM, "bad dimensions (need m, n >= 1)");
    if (!rowptr || !colidx || !counts || (matrix != 0 && matrix != 1))
        return fail(nullptr, HPRLP_EINVAL, "bad argument");
    hprlp_options o;
    if (opt) o = *opt;
    else hprlp_default_options(&o);
    resolve_options(o);
    std::string err;
    if (int rc = validate_options(o, err)) return fail(nullptr, rc, err);
    if (rowptr[0] != 0) return fail(nullptr, HPRLP_EINVAL, "rowptr[0] must be 0");
    for (int64_t i = 0; i < m; ++i)
        if (rowptr[i + 1] < rowptr[i]) return fail(nullptr, HPRLP_EINVAL, "rowptr not monotone");
    for (int64_t p = 0; p < rowptr[m]; ++p)
        if (colidx[p] < 0 || colidx[p] >= n) return fail(nullptr, HPRLP_EINVAL, "column index out of range");
    std::vector<Bundle> bA, bT;
    std::vector<int64_t> rpT;
    detect_bundles(o, m, n, rowptr, colidx, nullptr, nullptr, bA, bT, &rpT);
    if (matrix == 1 && rpT.empty()) {  // the column counts, in the order create uses
        std::vector<int64_t> deg((size_t)n, 0);
        for (int64_t p = 0; p < rowptr[m]; ++p) deg[colidx[p]]++;
        if (o.reorder) std::stable_sort(deg.begin(), deg.end(), std::greater<int64_t>());
        rpT.assign((size_t)n + 1, 0);
        for (int64_t j = 0; j < n; ++j) rpT[j + 1] = rpT[j] + deg[j];
    }
    const ScheduleParams sp{o.tile_nnz, o.tile_rows, o.short_max, o.split_len, o.chunk_nnz};
    Schedule S;
    if (matrix == 0) build_schedule(m, rowptr, sp, nullptr, bA, S);
    else build_schedule(n, rpT.data(), sp, nullptr, bT, S);
    counts[0] = (int64_t)S.items.size(); counts[1] = S.n_tiles; counts[2] = S.n_rowitems;
    counts[3] = S.n_chunks; counts[4] = 0; counts[5] = S.n_bundle_items;
    return HPRLP_OK;
}

extern "C" int hprlp_workspace_bytes_batched(int32_t n_inst, int64_t m, int64_t n, int64_t nnz,
                                             const hprlp_options *opt, size_t *bytes) {
    if (opt && opt->t1_zero) return fail(nullptr, HPRLP_EINVAL, "t1_zero applies to single LPs");
    return workspace_impl(n_inst, m, n, nnz, opt, bytes, true);
}

extern "C" int hprlp_create(hprlp_handle **out, int64_t m1, int64_t m2, int64_t n,
                            const int64_t *rowptr, const int32_t *colidx, const double *val,
                            const double *b, const double *c, const double *l, const double *u,
                            const hprlp_options *opt, void *d_workspace, size_t ws_bytes,
                            void *stream) {
    if (!out) return fail(nullptr, HPRLP_EINVAL, "out is null");
    *out = nullptr;
    if (m1 < 0 || m2 < 0 || m1 + m2 < 1 || n < 1)
        return fail(nullptr, HPRLP_EDIM, "bad dimensions (need m1, m2 >= 0, m1 + m2 >= 1, n >= 1)");
    Layout L{1, {0, m1 + m2}, {0, n}, {m1}, false};
    return create_impl(out, L, rowptr, colidx, val, b, c, l, u, nullptr, opt, d_workspace,
                       ws_bytes, stream);
}

extern "C" int hprlp_create_noalloc(hprlp_handle **out, int64_t m1, int64_t m2, int64_t n,
                                    const int64_t *rowptr, const int32_t *colidx,
                                    const double *val, const double *b, const double *c,
                                    const double *l, const double *u,
                                    const hprlp_options *opt, void *stream) {
    if (!out) return fail(nullptr, HPRLP_EINVAL, "out is null");
    *out = nullptr;
    if (m1 < 0 || m2 < 0 || m1 + m2 < 1 || n < 1)
        return fail(nullptr, HPRLP_EDIM, "bad dimensions (need m1, m2 >= 0, m1 + m2 >= 1, n >= 1)");
    if (!rowptr) return fail(nullptr, HPRLP_EINVAL, "rowptr is null");
    hprlp_options o;
    if (opt) o = *opt;
    else hprlp_default_options(&o);
    // nothing that allocates: no captured graphs, no timing events, no autotuner trials
    if (o.profile != 0 || o.autotune != 0)
        return fail(nullptr, HPRLP_EINVAL, "hprlp_create_noalloc needs profile = 0 and autotune = 0");
    o.graph = 0;
    const int64_t m = m1 + m2;
    if (rowptr[m] < 1) return fail(nullptr, HPRLP_EDIM, "A has no nonzero");
    size_t need = 0;
    int rc = hprlp_workspace_bytes(m1, m2, n, rowptr[m], &o, &need);
    if (rc) return rc;
    if (need > kScratchBytes)
        return fail(nullptr, HPRLP_EINVAL, "problem needs " + std::to_string(need) +
                                               " workspace bytes, above the static scratch of " +
                                               std::to_string(kScratchBytes));
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices)
        return fail(nullptr, HPRLP_EHIP, "hipGetDevice failed");
    void *ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_scratch_mu);
        if (g_scratch_owner[dev])
            return fail(nullptr, HPRLP_ESTATE, "the static scratch of this device is in use by "
                                               "a live hprlp_create_noalloc handle");
        if (!g_scratch_ptr[dev]) {
            const hipError_t e = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
            if (e != hipSuccess || !g_scratch_ptr[dev]) {
                g_scratch_ptr[dev] = nullptr;
                return fail(nullptr, HPRLP_EHIP, std::string("hipGetSymbolAddress(scratch): ") +
                                                     hipGetErrorString(e));
            }
        }
        ptr = g_scratch_ptr[dev];
        Layout L{1, {0, m}, {0, n}, {m1}, false};
        rc = create_impl(out, L, rowptr, colidx, val, b, c, l, u, nullptr, &o, ptr,
                         kScratchBytes, stream, true);
        if (rc == HPRLP_OK) g_scratch_owner[dev] = *out;
    }
    return rc;
}

extern "C" int hprlp_create_batched(hprlp_handle **out, int32_t n_inst,
                                    const int64_t *inst_row_off, const int64_t *inst_col_off,
                                    const int64_t *inst_m1, const int64_t *rowptr,
                                    const int32_t *colidx, const double *val, const double *b,
                                    const double *c, const double *l, const double *u,
                                    const double *lambda_inst, const hprlp_options *opt,
                                    void *d_workspace, size_t ws_bytes, void *stream) {
    if (!out || !inst_row_off || !inst_col_off || !inst_m1)
        return fail(nullptr, HPRLP_EINVAL, "null argument");
    *out = nullptr;
    if (n_inst < 1) return fail(nullptr, HPRLP_EDIM, "n_inst must be >= 1");
    Layout L;
    L.n_inst = n_inst;
    L.batched = true;
    L.row_off.assign(inst_row_off, inst_row_off + n_inst + 1);
    L.col_off.assign(inst_col_off, inst_col_off + n_inst + 1);
    L.m1.assign(inst_m1, inst_m1 + n_inst);
    if (L.row_off[n_inst] < 1 || L.col_off[n_inst] < 1 || L.row_off[n_inst] >= (1LL << 31) ||
        L.col_off[n_inst] >= (1LL << 31))
        return fail(nullptr, HPRLP_EDIM, "bad dimensions");
    return create_impl(out, L, rowptr, colidx, val, b, c, l, u, lambda_inst, opt, d_workspace,
                       ws_bytes, stream);
}

namespace {

// Halpern weights of Algorithm 2 at inner counter t (before it is incremented).
void fill_scalars(const hprlp_handle *h, IterScalars &s) {
    const double t = (double)h->t;
    s.sigma = h->sigma;
    s.lam_sigma = h->lambda * h->sigma;
    if (h->opt.use_halpern) {
        s.hx0 = 1.0 / (t + 1.0);
        s.hx1 = t / (t + 1.0);
        s.hy0 = 1.0 / (t + 2.0);
        s.hy1 = (t + 1.0) / (t + 2.0);
    } else {
        s.hx0 = 0.0; s.hx1 = 1.0; s.hy0 = 0.0; s.hy1 = 1.0;
    }
    s.m1 = h->m1;
    s.rho = h->opt.rho;
}

// Vectors of the passes: the displacement set in the FP32 phase of MIXED, else the FP64 set.
const void *pass_set(const hprlp_handle *h, int prec) {
    return prec == 1 ? static_cast<const void *>(&h->vdisp) : static_cast<const void *>(&h->v64);
}
const void *cur_set(const hprlp_handle *h) { return pass_set(h, h->prec); }
// The checks always run on FP64 vectors (prec 0 or 2): in the FP32 phase the iterations that
// keep w_bar write it in FP64.
int check_prec(int prec) { return prec == 1 ? 2 : prec; }

BatchArgs batch_args(const hprlp_handle *h, int iter_off) {
    BatchArgs a;
    a.sigma = h->bd.sigma;
    a.lam = h->bd.lam;
    a.kstart = h->bd.kstart;
    a.kbase = h->bd.kbase;
    a.m1_end = h->bd.m1_end;
    a.active = h->bd.active;
    a.inv_norm = h->bd.inv_norm;
    a.iter_off = iter_off;
    a.halpern = h->opt.use_halpern;
    a.rho = h->opt.rho;
    return a;
}

struct ProfRec {
    size_t ev0;  // events ev0 (before), ev0+1 (after the main kernel), ev0+2 (after finisher)
    bool col;
};

// One iteration (column pass then row pass).  keep: also store w_bar and d = w - w_hat.
// y-step of one iteration: the row pass (eq. update-y-2), or with T1 = 0 the exact solve
hipError_t row_step(hprlp_handle *h, bool keep, const IterScalars &s, const void *vs,
                    hipEvent_t em) {
    if (!h->opt.t1_zero) return launch_row_pass(h->prec, keep, h->A, vs, s, h->st, em);
    hipError_t e = t1_row_step(h->A, h->v64, s, h->t1.G, h->t1.r, h->t1.P, (int)h->m, keep,
                               h->st);
    if (e == hipSuccess && em) e = hipEventRecord(em, h->st);
    return e;
}

int run_iteration(hprlp_handle *h, bool keep, std::vector<ProfRec> *prof, size_t *ev_next) {
    IterScalars s;
    fill_scalars(h, s);
    const void *vs = cur_set(h);
    for (int pass = 0; pass < 2; ++pass) {
        hipEvent_t e0 = nullptr, em = nullptr, e1 = nullptr;
        if (prof) {
            e0 = pool_event(h, *ev_next);
            em = pool_event(h, *ev_next + 1);
            e1 = pool_event(h, *ev_next + 2);
            if (!e0 || !em || !e1) return fail(h, HPRLP_EHIP, "hipEventCreate failed");
            prof->push_back({*ev_next, pass == 0});
            *ev_next += 3;
            HIPCHK(h, hipEventRecord(e0, h->st));
        }
        hipError_t e = pass == 0 ? launch_col_pass(h->prec, keep, h->T, vs, s, h->st, em)
                                 : row_step(h, keep, s, vs, em);
        if (e != hipSuccess) return fail(h, HPRLP_EHIP, std::string("pass launch: ") + hipGetErrorString(e));
        if (prof) HIPCHK(h, hipEventRecord(e1, h->st));
    }
    h->t += 1;
    h->k += 1;
    return HPRLP_OK;
}

int run_check(hprlp_handle *h, int slot) {
    double *outr = h->res + (size_t)(2 * slot) * kNQ;
    double *outc = outr + kNQ;
    const int cp = check_prec(h->prec);
    hipError_t e = launch_check_row(cp, h->A, pass_set(h, cp), h->chk, h->v64.bd, h->m1,
                                    h->partsA, outr, h->st);
    if (e == hipSuccess)
        e = launch_check_col(cp, h->T, pass_set(h, cp), h->chk, h->v64.cd, h->v64.sc, h->partsT,
                             outc, h->st);
    if (e == hipSuccess && h->opt.t1_zero) {
        // T1 = 0: the y block of M is sigma A~A~^T, so the merit's ||dy||^2 becomes
        // ||A~^T dy||^2, and Delta_y of eq. sigma_T1=0 is ||A~^T (y_bar - y0)|| (lambda = 1)
        e = t1_atv_sq(h->T, (int)h->n, h->v64.dy, nullptr, h->t1.parts, outr + 3, h->st);
        if (e == hipSuccess)
            e = t1_atv_sq(h->T, (int)h->n, h->v64.ybar, h->v64.y0, h->t1.parts, outr + 5, h->st);
    }
    if (e != hipSuccess) return fail(h, HPRLP_EHIP, std::string("check launch: ") + hipGetErrorString(e));
    return HPRLP_OK;
}

double merit_of(const double *q, double sigma, double lambda) {
    // ||w - w_hat||_M^2 = sigma lambda ||dy||^2 + 2 <dy, A~ dx> + ||dx||^2 / sigma
    const double v = sigma * lambda * q[3] + 2.0 * q[4] + q[kNQ + 4] / sigma;
    return std::sqrt(v > 0.0 ? v : 0.0);
}

int set_schedules(hprlp_handle *h, const std::vector<int> &keep);

// Power method (Section 4.1) on every instance at once: v0 = 1/sqrt(m_b) on the rows of
// instance b; lambda_b is the Rayleigh quotient at the first iteration whose change is
// <= power_tol relative (or at power_max_iter).  Writes lam[b] and the largest iteration
// count over the instances.
int power_method(hprlp_handle *h, std::vector<double> &lam, int *iters) {
    const int64_t m = h->m;
    const int ni = h->n_inst;
    const std::vector<int64_t> &roff = h->row_off;
    std::vector<double> v0((size_t)m);
    for (int b = 0; b < ni; ++b)
        for (int64_t i = roff[b]; i < roff[b + 1]; ++i)
            v0[i] = (1.0 / std::sqrt((double)(roff[b + 1] - roff[b]))) *
                    (h->mixed ? h->dr[i] : 1.0);
    int rc = upload(h, h->vg, v0.data(), (size_t)m);
    if (rc) return rc;
    std::vector<double> ones((size_t)ni, 1.0);
    if ((rc = upload(h, h->inv_norm, ones.data(), (size_t)ni))) return rc;
    const BatchArgs ba = batch_args(h, 0);
    const int maxit = h->opt.power_max_iter;
    const double tol = h->opt.power_tol;
    std::vector<double> rq_prev((size_t)ni, 0.0);
    std::vector<int> done((size_t)ni, 0);
    lam.assign((size_t)ni, 0.0);
    int n_done = 0, max_it = 0;
    const int B = 32;
    for (int k0 = 0; k0 < maxit && n_done < ni; k0 += B) {
        const int kb = std::min(B, maxit - k0);
        for (int kk = 0; kk < kb; ++kk) {
            hipError_t e = launch_power_iter(
                h->mixed, h->mixed, h->A, h->T, h->vg, h->w, h->v64.sc, h->v64.sr, h->inv_norm,
                h->partsT, h->partsA, h->hist, k0 + kk, h->st, h->batched ? &ba : nullptr,
                h->batched ? &h->segA : nullptr, h->batched ? &h->segT : nullptr,
                h->batched ? h->bd.seg_tmp : nullptr);
            if (e != hipSuccess) return fail(h, HPRLP_EHIP, std::string("power launch: ") + hipGetErrorString(e));
        }
        if ((rc = download(h, h->pinned, h->hist + (size_t)k0 * ni, (size_t)kb * ni))) return rc;
        for (int b = 0; b < ni; ++b) {
            if (done[b]) continue;
            for (int kk = 0; kk < kb; ++kk) {
                const int it = k0 + kk + 1;
                const double rq = h->pinned[(size_t)kk * ni + b];
                lam[b] = rq;
                if ((it > 1 && std::fabs(rq - rq_prev[b]) <= tol * rq) || it == maxit) {
                    done[b] = it;
                    break;
                }
                rq_prev[b] = rq;
            }
            if (done[b]) {
                n_done++;
                max_it = std::max(max_it, done[b]);
            }
        }
        if (h->batched && n_done < ni) {
            // instances whose lambda is settled leave the schedules once they hold an eighth
            // of the scheduled nonzeros (the others' iterations are unchanged)
            int64_t live = 0;
            for (int b = 0; b < ni; ++b)
                if (!done[b]) live += h->inst_nnz[b];
            if (live <= (h->sched_nnz * 7) / 8) {
                std::vector<int> keep((size_t)ni);
                for (int b = 0; b < ni; ++b) keep[b] = done[b] ? 0 : 1;
                if ((rc = set_schedules(h, keep))) return rc;
            }
        }
    }
    *iters = max_it;
    if (h->batched && h->compacted && (rc = set_schedules(h, {}))) return rc;
    return HPRLP_OK;
}

int zero_state(hprlp_handle *h) {
    const long long n = h->n, m = h->m;
    hipError_t e = hipSuccess;
    if (h->prec == 1) {  // anchors at the origin, zero displacements, the anchor's data
        for (double *p : {h->v64.x0, h->v64.xbar})
            if (e == hipSuccess) e = launch_fill(p, n, 0.0, h->st);
        for (double *p : {h->v64.y0, h->v64.ybar})
            if (e == hipSuccess) e = launch_fill(p, m, 0.0, h->st);
        for (float *p : {h->vdisp.dxh, h->vdisp.dxrel})
            if (p && e == hipSuccess) e = launch_fill_f(p, n, 0.f, h->st);
        if (e == hipSuccess) e = launch_fill_f(h->vdisp.dy, m, 0.f, h->st);
        if (e == hipSuccess) e = launch_anchor(h->A, h->T, h->vdisp, h->st);
    } else {
        for (double *p : {h->v64.xhat, h->v64.x0, h->v64.xrel})
            if (p && e == hipSuccess) e = launch_fill(p, n, 0.0, h->st);
        for (double *p : {h->v64.y, h->v64.y0})
            if (e == hipSuccess) e = launch_fill(p, m, 0.0, h->st);
    }
    if (e != hipSuccess) return fail(h, HPRLP_EHIP, hipGetErrorString(e));
    return HPRLP_OK;
}

// w^{r+1,0} = w_bar: anchors and current iterate (x is rebuilt from x_hat and x0).
int restart_copy(hprlp_handle *h) {
    const long long n = h->n, m = h->m;
    hipError_t e;
    if (h->prec == 1) {  // FP32 phase: the anchor moves to w_bar, its data is renewed
        e = launch_reanchor(h->vdisp, n, m, h->st);
        if (e == hipSuccess) e = launch_anchor(h->A, h->T, h->vdisp, h->st);
    } else {
        e = launch_copy_d(h->v64.x0, h->v64.xbar, n, h->st);
        if (e == hipSuccess) e = launch_copy_d(h->v64.xhat, h->v64.xbar, n, h->st);
        if (e == hipSuccess && h->v64.xrel) e = launch_copy_d(h->v64.xrel, h->v64.xbar, n, h->st);
        if (e == hipSuccess) e = launch_copy_d(h->v64.y0, h->v64.ybar, m, h->st);
        if (e == hipSuccess) e = launch_copy_d(h->v64.y, h->v64.ybar, m, h->st);
    }
    if (e != hipSuccess) return fail(h, HPRLP_EHIP, hipGetErrorString(e));
    return HPRLP_OK;
}

// MIXED: continue in FP64 from the FP32 phase's state: x_hat, x_rel and y become anchor +
// displacement; the anchors and the last w_bar (x_bar, z, dx, y_bar, dy) are FP64 already.
int promote(hprlp_handle *h) {
    const hipError_t e = launch_disp_promote(h->vdisp, h->n, h->m, h->st);
    if (e != hipSuccess) return fail(h, HPRLP_EHIP, hipGetErrorString(e));
    h->prec = 2;
    return HPRLP_OK;
}

int copy_out(hprlp_handle *h, double *dst, const double *src, long long k) {
    if (!dst || k == 0) return HPRLP_OK;
    HIPCHK(h, hipMemcpyAsync(dst, src, (size_t)k * sizeof(double), hipMemcpyDefault, h->st));
    HIPCHK(h, hipStreamSynchronize(h->st));
    return HPRLP_OK;
}

// w_bar of the last check, original space, into x, y, z (host or device pointers).
int write_outputs(hprlp_handle *h, double *x, double *y, double *z) {
    const bool f32 = false;  // w_bar is kept in FP64 in every phase
    const void *xb = f32 ? (const void *)h->v32.xbar : (const void *)h->v64.xbar;
    const void *yb = f32 ? (const void *)h->v32.ybar : (const void *)h->v64.ybar;
    const void *zb = f32 ? (const void *)h->v32.zint : (const void *)h->v64.zint;
    double *ox = h->outv, *oy = h->outv + h->n, *oz = h->outv + h->n + h->m;
    hipError_t e = launch_scale_out(ox, xb, f32, h->ux, 0.0, h->cperm, h->n, h->st);
    if (e == hipSuccess) e = launch_scale_out(oy, yb, f32, h->uy, 0.0, nullptr, h->m, h->st);
    if (e == hipSuccess) e = launch_scale_out(oz, zb, f32, h->chk.co, 0.0, h->cperm, h->n, h->st);
    if (e != hipSuccess) return fail(h, HPRLP_EHIP, hipGetErrorString(e));
    HIPCHK(h, hipStreamSynchronize(h->st));
    int rc;
    if ((rc = copy_out(h, x, ox, h->n)) || (rc = copy_out(h, y, oy, h->m)) ||
        (rc = copy_out(h, z, oz, h->n)))
        return rc;
    return HPRLP_OK;
}

double bytes_per_iter(const hprlp_handle *h) {
    const double sv = h->mixed ? 4.0 : 8.0, svec = (h->prec == 1) ? 4.0 : 8.0;
    return 2.0 * h->nnz * (sv + 4.0) + 4.0 * (h->m + h->n + 2) + 7.0 * h->n * svec +
           5.0 * h->m * svec;
}

// Per-instance device state of a batched solve at its start: every instance iterates from
// k = 0 with sigma = sigma0 (lambda is set after the power method).
int init_batch_state(hprlp_handle *h, double sigma0, double lam) {
    const int ni = h->n_inst;
    std::vector<double> sig((size_t)ni, sigma0), lamv((size_t)ni, lam), zeros((size_t)ni, 0.0);
    std::vector<long long> zl((size_t)ni, 0);
    std::vector<int> ones((size_t)ni, 1), zi((size_t)ni, 0);
    const long long kb0 = 0;
    int rc;
    if ((rc = upload(h, h->bd.sigma, sig.data(), sig.size())) ||
        (rc = upload(h, h->bd.lam, lamv.data(), lamv.size())) ||
        (rc = upload(h, h->bd.merit0, zeros.data(), zeros.size())) ||
        (rc = upload(h, h->bd.merit_prev, zeros.data(), zeros.size())) ||
        (rc = upload(h, h->bd.kstart, zl.data(), zl.size())) ||
        (rc = upload(h, h->bd.kbase, &kb0, 1)) ||
        (rc = upload(h, h->bd.iters_done, zl.data(), zl.size())) ||
        (rc = upload(h, h->bd.restarts, zl.data(), zl.size())) ||
        (rc = upload(h, h->bd.nchecks, zl.data(), zl.size())) ||
        (rc = upload(h, h->bd.active, ones.data(), ones.size())) ||
        (rc = upload(h, h->bd.status, zi.data(), zi.size())) ||
        (rc = upload(h, h->bd.restart_flag, zi.data(), zi.size())))
        return rc;
    return HPRLP_OK;
}

// Upload schedule S as the schedule of A (col = false) or A^T (col = true), with the
// per-instance slot lists of a batched handle.
int install_schedule(hprlp_handle *h, bool col, Schedule &&S) {
    DevMat &M = col ? h->T : h->A;
    const int *cap = col ? h->capT : h->capA;
    if ((int)S.items.size() > cap[0] || (int)S.splits.size() > cap[1] || S.n_chunk_slots > cap[2])
        return fail(h, HPRLP_ESTATE, "schedule exceeds the carved capacity");
    HIPCHK(h, hipStreamSynchronize(h->st));
    int rc;
    if ((rc = upload(h, M.items, S.items.data(), S.items.size())) ||
        (rc = upload(h, M.splits, S.splits.data(), S.splits.size())))
        return rc;
    M.n_items = (int)S.items.size();
    M.n_split = (int)S.splits.size();
    M.tile_nnz = S.tile_nnz;
    M.tile_rows = S.tile_rows;
    M.host = std::move(S);
    if (h->batched) {
        std::vector<int> ptr, slots;
        build_segments(M.host, h->n_inst, ptr, slots);
        if ((rc = upload(h, col ? h->bd.segT_ptr : h->bd.segA_ptr, ptr.data(), ptr.size())) ||
            (rc = upload(h, col ? h->bd.segT_slots : h->bd.segA_slots, slots.data(), slots.size())))
            return rc;
    }
    return HPRLP_OK;
}

// Mean duration (ms) of one launch of the row pass (col = false) or column pass, over
// kTuneReps launches after two warm-up launches, bracketed by HIP events.
// Time one pass as a solve runs it: every launch follows a launch of the other pass (the
// two matrices together outgrow the infinity cache, so back-to-back launches of one pass
// would find its matrix cached).  2 warm-up pairs, then kTuneReps pairs with HIP events
// around the pass being timed; the result is the mean of those launches.
int time_pass(hprlp_handle *h, bool col, double *ms) {
    IterScalars s;
    fill_scalars(h, s);
    const BatchArgs ba = batch_args(h, 0);
    const BatchArgs *pba = h->batched ? &ba : nullptr;
    const void *vs = cur_set(h);
    for (int i = 0; i < 2 * kTuneReps; ++i)
        if (!pool_event(h, (size_t)i)) return fail(h, HPRLP_EHIP, "hipEventCreate failed");
    for (int i = 0; i < 2 + kTuneReps; ++i) {
        for (int which = 0; which < 2; ++which) {
            const bool c = which == 0 ? !col : col;  // the other pass, then the timed one
            const bool timed = which == 1 && i >= 2;
            if (timed) HIPCHK(h, hipEventRecord(h->ev_pool[2 * (i - 2)], h->st));
            const hipError_t e = c ? launch_col_pass(h->prec, false, h->T, vs, s, h->st, nullptr, pba)
                                   : launch_row_pass(h->prec, false, h->A, vs, s, h->st, nullptr, pba);
            if (e != hipSuccess) return fail(h, HPRLP_EHIP, std::string("pass launch: ") + hipGetErrorString(e));
            if (timed) HIPCHK(h, hipEventRecord(h->ev_pool[2 * (i - 2) + 1], h->st));
        }
    }
    HIPCHK(h, hipEventSynchronize(h->ev_pool[2 * kTuneReps - 1]));
    double total = 0.0;
    for (int i = 0; i < kTuneReps; ++i) {
        float t = 0.f;
        HIPCHK(h, hipEventElapsedTime(&t, h->ev_pool[2 * i], h->ev_pool[2 * i + 1]));
        total += t;
    }
    *ms = total / kTuneReps;
    return HPRLP_OK;
}

// Tiles of A (row) and / or A^T (col) to column order (to_col) or back to row order.
int set_tile_order(hprlp_handle *h, bool row, bool col, bool to_col) {
    for (int w = 0; w < 2; ++w) {
        DevMat &M = w ? h->T : h->A;
        if (!(w ? col : row) || !M.pos || M.sorted == to_col) continue;
        const hipError_t e = launch_tile_order(M, h->mixed, to_col, h->st);
        if (e != hipSuccess) return fail(h, HPRLP_EHIP, std::string("tile order: ") + hipGetErrorString(e));
        M.sorted = to_col;
    }
    HIPCHK(h, hipStreamSynchronize(h->st));
    return HPRLP_OK;
}

bool same_schedule(const Schedule &a, const Schedule &b) {
    return a.items.size() == b.items.size() && a.splits.size() == b.splits.size() &&
           std::memcmp(a.items.data(), b.items.data(), a.items.size() * sizeof(int4)) == 0 &&
           std::memcmp(a.splits.data(), b.splits.data(), a.splits.size() * sizeof(int4)) == 0;
}

// Schedule autotuner: for each matrix, coordinate descent over the candidate table (tile
// shape, then short_max, then split_len x chunk_nnz when rows are long enough to split),
// timing the pass of each distinct schedule on the uploaded problem (Halpern state at the
// origin, sigma = lambda = 1).  A candidate replaces the best one only if it is at least 3%
// faster.  The chosen schedules stay installed; their parameters are in spA / spT.
int tune_schedules(hprlp_handle *h, const int64_t *rpA, const int64_t *rpT,
                   const int32_t *inst_row, const int32_t *inst_col) {
    int rc;
    h->prec = h->f32phase ? 1 : (h->mixed ? 2 : 0);
    h->t = 0;
    h->sigma = 1.0;
    h->lambda = 1.0;
    if ((rc = zero_state(h))) return rc;
    if (h->batched && (rc = init_batch_state(h, 1.0, 1.0))) return rc;
    for (int w = 0; w < 2; ++w) {
        const bool col = w == 1;
        const int64_t rows = col ? h->n : h->m;
        const int64_t *rp = col ? rpT : rpA;
        const int32_t *inst = col ? inst_col : inst_row;
        ScheduleParams best = col ? h->spT : h->spA;
        int64_t maxlen = 0;
        for (int64_t r = 0; r < rows; ++r) maxlen = std::max(maxlen, rp[r + 1] - rp[r]);
        Schedule cur = (col ? h->T : h->A).host;  // installed at create
        double best_ms = 0.0;
        if ((rc = time_pass(h, col, &best_ms))) return rc;
        Schedule best_s = cur;
        auto cap_ok = [&](const Schedule &S) {
            const int *cap = col ? h->capT : h->capA;
            return (int)S.items.size() <= cap[0] && (int)S.splits.size() <= cap[1] &&
                   S.n_chunk_slots <= cap[2];
        };
        // One coordinate of the descent: the candidate schedules are built on host threads
        // (pure functions of the row pointers), then installed and timed one by one.
        auto sweep = [&](const std::vector<ScheduleParams> &cands) -> int {
            std::vector<Schedule> built(cands.size());
            std::vector<char> ok(cands.size(), 0);
            std::atomic<size_t> next{0};
            auto worker = [&]() {
                for (size_t c; (c = next.fetch_add(1)) < cands.size();) {
                    const ScheduleParams &p = cands[c];
                    if (p.short_max > p.tile_nnz || p.split_len < p.short_max) continue;
                    build_schedule(rows, rp, p, inst, (col ? h->T : h->A).bundles, built[c]);
                    ok[c] = 1;
                }
            };
            const size_t nt = std::min<size_t>(cands.size(), 8);
            std::vector<std::thread> pool;
            for (size_t t = 1; t < nt; ++t) pool.emplace_back(worker);
            worker();
            for (auto &t : pool) t.join();
            for (size_t c = 0; c < cands.size(); ++c) {
                if (!ok[c] || !cap_ok(built[c]) || same_schedule(built[c], best_s)) continue;
                Schedule keep = built[c];
                int r2 = install_schedule(h, col, std::move(built[c]));
                if (r2) return r2;
                double ms = 0.0;
                if ((r2 = time_pass(h, col, &ms))) return r2;
                if (ms < 0.97 * best_ms) {
                    best_ms = ms;
                    best = cands[c];
                    best_s = std::move(keep);
                }
            }
            return HPRLP_OK;
        };
        {
            const ScheduleParams b0 = best;
            std::vector<ScheduleParams> c;
            for (int tn : kTuneTileNnz)
                for (int tr : kTuneTileRows)
                    c.push_back({tn, tr, std::min(b0.short_max, tn), b0.split_len, b0.chunk_nnz});
            if ((rc = sweep(c))) return rc;
        }
        {
            const ScheduleParams shape = best;
            std::vector<ScheduleParams> c;
            for (int sm : kTuneShortMax)
                c.push_back({shape.tile_nnz, shape.tile_rows, sm, std::max(shape.split_len, sm),
                             shape.chunk_nnz});
            if ((rc = sweep(c))) return rc;
        }
        if (maxlen > kTuneMinSplit) {
            const ScheduleParams sh = best;
            std::vector<ScheduleParams> c;
            for (int sl : kTuneSplitLen)
                for (int ch : kTuneChunk) c.push_back({sh.tile_nnz, sh.tile_rows, sh.short_max, sl, ch});
            if ((rc = sweep(c))) return rc;
        }
        if ((rc = install_schedule(h, col, std::move(best_s)))) return rc;
        (col ? h->spT : h->spA) = best;
        // the chosen schedule with its tiles in column order; kept only if >= 3% faster
        if ((col ? h->T : h->A).pos && h->opt.tile_order == -1) {
            if ((rc = set_tile_order(h, !col, col, true))) return rc;
            double ms = 0.0;
            if ((rc = time_pass(h, col, &ms))) return rc;
            if (ms < 0.97 * best_ms) best_ms = ms;
            else if ((rc = set_tile_order(h, !col, col, false))) return rc;
        }
        h->tuned_ms[w] = best_ms;
    }
    return HPRLP_OK;
}

// ---------------------------------------------------------------------------- one LP

// The plain iterations between two checks of one LP as a captured graph: `len` iterations of
// the instance-scalar passes (t = k_base + i - k_start, sigma and lambda read from device
// memory, as in a batch of one), then k_base += len.  Captured on a stream of the handle's
// own, launched on the handle's stream.
int single_graph(hprlp_handle *h, int prec, int len, hipGraphExec_t *out) {
    if (!h->graphs[prec]) {
        if (!h->cap_st)
            HIPCHK(h, hipStreamCreateWithFlags(&h->cap_st, hipStreamNonBlocking));
        const void *vs = pass_set(h, prec);
        const IterScalars unused{};
        HIPCHK(h, hipStreamBeginCapture(h->cap_st, hipStreamCaptureModeThreadLocal));
        hipError_t e = hipSuccess;
        for (int i = 0; i < len && e == hipSuccess; ++i) {
            const BatchArgs ba = batch_args(h, i);
            e = launch_col_pass(prec, false, h->T, vs, unused, h->cap_st, nullptr, &ba);
            if (e == hipSuccess)
                e = launch_row_pass(prec, false, h->A, vs, unused, h->cap_st, nullptr, &ba);
        }
        if (e == hipSuccess) e = launch_advance(h->bd.kbase, len, h->cap_st);
        hipGraph_t g = nullptr;
        const hipError_t e2 = hipStreamEndCapture(h->cap_st, &g);
        if (e != hipSuccess || e2 != hipSuccess) {
            if (g) (void)hipGraphDestroy(g);
            return fail(h, HPRLP_EHIP, std::string("chunk capture: ") +
                                           hipGetErrorString(e != hipSuccess ? e : e2));
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t e3 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e3 != hipSuccess) return fail(h, HPRLP_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e3));
        h->graphs[prec] = ex;
    }
    *out = h->graphs[prec];
    return HPRLP_OK;
}

// Below this many nonzeros a single LP's passes are launch-bound and the chunk graphs pay
// (measured: 8.6 -> 6.9 us per iteration at 1e3 nonzeros); at 1e6 nonzeros the launches
// are already hidden behind the kernels and the instance-scalar kernels cost more than they
// save (14.0 -> 15.2 us per iteration; zipf1m, 1.1e7 nonzeros: +4%).
constexpr int64_t kGraphMaxNnz = 100000;

// Run `count` plain iterations of one LP, whole chunks through the captured graph.
int run_plain(hprlp_handle *h, long long count) {
    const int len = (int)h->opt.check_every - 2;
    const bool use = h->opt.graph == 2 || (h->opt.graph == 1 && h->nnz < kGraphMaxNnz);
    if (use && len >= 1 && count >= len) {
        hipGraphExec_t ex;
        int rc = single_graph(h, h->prec, len, &ex);
        if (rc) return rc;
        // device scalars of this stretch (the staging slot follows the check results in the
        // pinned buffer; the stream is synchronised at every check, so it is free again)
        double *stage = h->pinned + 4 * kNQ;
        stage[0] = h->sigma;
        stage[1] = h->lambda;
        const long long ks = h->k - h->t, kb = h->k;
        std::memcpy(stage + 2, &ks, sizeof ks);
        std::memcpy(stage + 3, &kb, sizeof kb);
        HIPCHK(h, hipMemcpyAsync(h->bd.sigma, stage, 4 * sizeof(double), hipMemcpyHostToDevice, h->st));
        while (count >= len) {
            HIPCHK(h, hipGraphLaunch(ex, h->st));
            h->k += len;
            h->t += len;
            count -= len;
        }
    }
    size_t ev = 0;
    for (; count > 0; --count)
        if (int rc = run_iteration(h, false, nullptr, &ev)) return rc;
    return HPRLP_OK;
}

// Start of a single-LP solve: lambda (power method unless given; Section 4.1), sigma0 and
// the origin, with t = k = r = 0.  Returns with h->lambda <= 0 reported as NUMERICAL.
int single_begin(hprlp_handle *h, int *status, int *piters) {
    const hprlp_options &o = h->opt;
    h->solved = false;  // outputs of an earlier solve are no longer the handle's
    h->trace.clear();
    h->stats = hprlp_stats_t{};
    h->prec = h->f32phase ? 1 : (h->mixed ? 2 : 0);
    h->t = h->k = h->r = 0;
    h->sigma = o.sigma0;
    int rc;
    *piters = 0;
    if (o.t1_zero) {
        h->lambda = 1.0;  // no lambda in this variant; 1 leaves the merit and Delta_y as above
    } else if (o.lambda_override > 0) {
        h->lambda = o.lambda_override;
    } else {
        std::vector<double> lam;
        if ((rc = power_method(h, lam, piters))) return rc;
        h->lambda = lam[0];
    }
    if (!(h->lambda > 0.0) || !std::isfinite(h->lambda)) {
        h->stats.status = HPRLP_NUMERICAL;
        if (status) *status = HPRLP_NUMERICAL;
        return fail(h, HPRLP_OK, "power method gave lambda <= 0");
    }
    return zero_state(h);
}

int solve_single(hprlp_handle *h, double *x, double *y, double *z, int *status) {
    const hprlp_options &o = h->opt;
    HIPCHK(h, hipStreamSynchronize(h->st));
    const double t_start = now_ms();
    int rc;
    int piters = 0;
    if ((rc = single_begin(h, status, &piters))) return rc;
    if (h->stats.status == HPRLP_NUMERICAL) return HPRLP_OK;
    const double t_power = now_ms() - t_start;

    std::vector<ProfRec> prof;
    size_t ev_next = 0;
    std::vector<ProfRec> *pp = o.profile ? &prof : nullptr;
    double prof_ms[2] = {0, 0}, split_ms = 0;
    long long prof_n[2] = {0, 0};
    auto flush_prof = [&]() -> int {
        for (auto &p : prof) {
            float ms = 0, ms2 = 0;
            HIPCHK(h, hipEventElapsedTime(&ms, h->ev_pool[p.ev0], h->ev_pool[p.ev0 + 1]));
            HIPCHK(h, hipEventElapsedTime(&ms2, h->ev_pool[p.ev0 + 1], h->ev_pool[p.ev0 + 2]));
            prof_ms[p.col ? 0 : 1] += ms;
            prof_n[p.col ? 0 : 1] += 1;
            split_ms += ms2;
        }
        prof.clear();
        ev_next = 0;
        return HPRLP_OK;
    };

    double merit0 = 0, merit_prev = 0;
    bool pending_first = false;
    std::vector<double> kkt_hist;  // MIXED: rel. KKT at the checks of the FP32 phase
    int st_out = HPRLP_UNSOLVED;
    long long iters_fp32 = 0;
    const long long ce = o.check_every;
    for (;;) {
        const bool first = h->t == 0;
        const long long kn = h->k + 1;
        const bool chk = (kn % ce == 0) || kn >= o.max_iter;
        if (!first && !chk) {
            const long long next_check = ((h->k / ce) + 1) * ce;
            const long long last = std::min(next_check, o.max_iter) - 1;
            if (!pp) {  // chunk graphs (option graph)
                if ((rc = run_plain(h, last - h->k))) return rc;
                continue;
            }
            while (h->k + 1 <= last) {
                // profile = N: bracket every N-th iteration's passes with HIP events
                const bool samp = (h->k % o.profile) == 0;
                if ((rc = run_iteration(h, false, samp ? pp : nullptr, &ev_next))) return rc;
            }
            continue;
        }
        if ((rc = run_iteration(h, true, nullptr, &ev_next))) return rc;
        if (h->prec == 1) iters_fp32 = h->k;
        if ((rc = run_check(h, chk ? 1 : 0))) return rc;
        if (!chk) {
            pending_first = true;
            continue;
        }
        HIPCHK(h, hipMemcpyAsync(h->pinned, h->res, 4 * kNQ * sizeof(double),
                                 hipMemcpyDeviceToHost, h->st));
        HIPCHK(h, hipStreamSynchronize(h->st));
        if (pp && (rc = flush_prof())) return rc;
        const double *q0 = h->pinned;            // first iteration of this outer loop
        const double *q = h->pinned + 2 * kNQ;   // this check
        const double merit = merit_of(q, h->sigma, h->lambda);
        if (pending_first) {
            merit0 = merit_of(q0, h->sigma, h->lambda);
            merit_prev = merit0;
            pending_first = false;
        }
        if (first) {
            merit0 = merit;
            merit_prev = merit;
        }
        const double bbc = h->beta_b * h->beta_c;
        const double rel_p = std::sqrt(q[0]) / (1.0 + h->bnorm);
        const double rel_d = std::sqrt(q[kNQ + 0]) / (1.0 + h->cnorm);
        const double pobj = bbc * q[kNQ + 2];
        const double dobj = bbc * q[2] - q[kNQ + 3];
        const double rel_gap = std::fabs(dobj - pobj) / (1.0 + std::fabs(dobj) + std::fabs(pobj));
        const double kkt = std::max(rel_gap, std::max(rel_p, rel_d));
        std::array<double, TR_NCOL> row{};
        row[TR_K] = (double)h->k; row[TR_T] = (double)h->t; row[TR_R] = (double)h->r;
        row[TR_SIGMA] = h->sigma; row[TR_MERIT] = merit; row[TR_MERIT0] = merit0;
        row[TR_MERIT_PREV] = merit_prev; row[TR_REL_P] = rel_p; row[TR_REL_D] = rel_d;
        row[TR_REL_GAP] = rel_gap; row[TR_POBJ] = pobj; row[TR_DOBJ] = dobj;
        row[TR_SIGMA_NEW] = h->sigma;
        h->stats.rel_p = rel_p; h->stats.rel_d = rel_d; h->stats.rel_gap = rel_gap;
        h->stats.pobj = pobj; h->stats.dobj = dobj;
        if (o.verbose)
            std::fprintf(stderr, "hprlp k=%lld r=%lld t=%lld sigma=%.3e p=%.2e d=%.2e g=%.2e merit=%.3e/%.3e\n",
                         h->k, h->r, h->t, h->sigma, rel_p, rel_d, rel_gap, merit, merit0);
        const double elapsed_s = (now_ms() - t_start) / 1000.0;
        if (!(kkt == kkt)) st_out = HPRLP_NUMERICAL;
        else if (kkt <= o.tol) st_out = HPRLP_OPTIMAL;
        else if (h->k >= o.max_iter) st_out = HPRLP_ITER_LIMIT;
        else if (o.time_limit > 0 && elapsed_s >= o.time_limit) st_out = HPRLP_TIME_LIMIT;
        if (st_out != HPRLP_UNSOLVED) {
            h->trace.push_back(row);
            break;
        }
        // ---- restart criteria (Section 3.1)
        bool restart = false;
        if (o.use_restart) {
            if (merit <= o.alpha1 * merit0) restart = true;
            if (merit <= o.alpha2 * merit0 && merit > merit_prev) restart = true;
            if ((double)h->t >= o.alpha3 * (double)h->k) restart = true;
        }
        if (restart) {
            double sig_new = h->sigma;
            if (o.sigma_update) {  // Algorithm 3 with eq. sigma_T1!=0
                const double Dx = std::sqrt(q[kNQ + 5]);
                const double Dy = std::sqrt(h->lambda) * std::sqrt(q[5]);
                const double err_p = std::sqrt(q[1]) / (1.0 + h->bsnorm);
                const double err_d = std::sqrt(q[kNQ + 1]) / (1.0 + h->csnorm);
                const bool ok = Dx > 1e-16 && Dx < 1e12 && Dy > 1e-16 && Dy < 1e12 &&
                                err_p > 0.0 && err_d / err_p > 1e-8 && err_d / err_p < 1e8;
                sig_new = ok ? Dx / Dy : 1.0;
                row[TR_DX] = Dx; row[TR_DY] = Dy; row[TR_ERR_P] = err_p; row[TR_ERR_D] = err_d;
            }
            row[TR_RESTART] = 1.0;
            row[TR_SIGMA_NEW] = sig_new;
            h->sigma = sig_new;
            if ((rc = restart_copy(h))) return rc;
            h->t = 0;
            h->r += 1;
        } else {
            merit_prev = merit;
        }
        h->trace.push_back(row);
        if (h->prec == 1) {
            // switch to FP64 at tol_switch, or (stall_checks > 0) when the iteration stalls: the
            // best residual of the last stall_checks checks is not below stall_ratio times
            // the best one before them
            bool sw = kkt <= o.tol_switch;
            kkt_hist.push_back(kkt);
            const size_t S = (size_t)o.stall_checks, H = kkt_hist.size();
            if (!sw && S > 0 && H > S) {
                const double before = *std::min_element(kkt_hist.begin(), kkt_hist.end() - S);
                const double recent = *std::min_element(kkt_hist.end() - S, kkt_hist.end());
                sw = recent > o.stall_ratio * before;
            }
            if (sw && (rc = promote(h))) return rc;
        }
    }
    HIPCHK(h, hipStreamSynchronize(h->st));
    if (pp && (rc = flush_prof())) return rc;
    const double t_end = now_ms();
    if ((rc = write_outputs(h, x, y, z))) return rc;
    h->solved = true;
    hprlp_stats_t &s = h->stats;
    s.iters = h->k;
    s.restarts = h->r;
    s.iters_fp32 = h->f32phase ? iters_fp32 : 0;
    s.status = st_out;
    s.power_iters = piters;
    s.sigma = h->sigma;
    s.lambda = o.t1_zero ? 0.0 : h->lambda;
    s.beta_b = h->beta_b;
    s.beta_c = h->beta_c;
    s.t_power_ms = t_power;
    s.t_solve_ms = t_end - t_start;
    s.bytes_per_iter = bytes_per_iter(h);
    s.col_pass_ms = prof_ms[0];
    s.row_pass_ms = prof_ms[1];
    s.col_pass_launches = prof_n[0];
    s.row_pass_launches = prof_n[1];
    s.split_ms = split_ms;
    s.n_checks = (long long)h->trace.size();
    s.t_setup_ms = h->t_setup_ms;
    s.t_prep_ms = h->t_prep_ms;
    s.t_tune_ms = h->t_tune_ms;
    if (status) *status = st_out;
    return HPRLP_OK;
}

// ---------------------------------------------------------------------------- a batch

// Rebuild the schedules of A and A^T over the instances with keep[b] != 0 (every instance
// when keep is empty), upload them with the per-instance slot lists, and drop the captured
// chunk graphs (they hold the old item counts).  Each instance's work items are the same as
// in the full schedule (tiles never straddle instances), so the result fits the carved
// arrays; stopped instances simply have no work item left.
int set_schedules(hprlp_handle *h, const std::vector<int> &keep) {
    int64_t nnz = h->nnz;
    if (!keep.empty()) {
        nnz = 0;
        for (int b = 0; b < h->n_inst; ++b)
            if (keep[b]) nnz += h->inst_nnz[b];
    }
    Schedule sa, stt;
    if (keep.empty()) {
        sa = h->A.full;
        stt = h->T.full;
    } else {
        filter_schedule(h->A.full, keep, sa);
        filter_schedule(h->T.full, keep, stt);
    }
    if ((int)sa.items.size() > h->capA[0] || (int)sa.splits.size() > h->capA[1] ||
        sa.n_chunk_slots > h->capA[2] || (int)stt.items.size() > h->capT[0] ||
        (int)stt.splits.size() > h->capT[1] || stt.n_chunk_slots > h->capT[2])
        return fail(h, HPRLP_ESTATE, "rebuilt schedule exceeds the carved capacity");
    int rc;
    if ((rc = install_schedule(h, false, std::move(sa))) || (rc = install_schedule(h, true, std::move(stt))))
        return rc;
    for (hipGraphExec_t &g : h->graphs)
        if (g) {
            (void)hipGraphExecDestroy(g);
            g = nullptr;
        }
    h->sched_nnz = nnz;
    h->compacted = !keep.empty();
    return HPRLP_OK;
}

// A chunk graph with event nodes.  Stream capture does not turn an event record into a
// graph node here, so the graph is assembled by hand: the launches between two marks are
// captured into a segment graph, appended as a child node, and each mark appends an event
// record node; all nodes form one chain, in launch order.
struct ChunkBuilder {
    hipStream_t st;
    hipGraph_t g = nullptr;
    hipGraphNode_t last = nullptr;
    bool capturing = false;
    hipError_t start() {
        hipError_t e = hipGraphCreate(&g, 0);
        if (e == hipSuccess) e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
        capturing = e == hipSuccess;
        return e;
    }
    // end the open capture and append its graph (if it has nodes) as a child node
    hipError_t close_segment() {
        hipGraph_t seg = nullptr;
        hipError_t e = hipStreamEndCapture(st, &seg);
        capturing = false;
        if (e != hipSuccess) return e;
        size_t nn = 0;
        e = hipGraphGetNodes(seg, nullptr, &nn);
        if (e == hipSuccess && nn > 0) {
            hipGraphNode_t node = nullptr;
            e = hipGraphAddChildGraphNode(&node, g, last ? &last : nullptr, last ? 1 : 0, seg);
            if (e == hipSuccess) last = node;
        }
        (void)hipGraphDestroy(seg);
        return e;
    }
    hipError_t mark(hipEvent_t ev) {
        hipError_t e = close_segment();
        hipGraphNode_t node = nullptr;
        if (e == hipSuccess)
            e = hipGraphAddEventRecordNode(&node, g, last ? &last : nullptr, last ? 1 : 0, ev);
        if (e == hipSuccess) {
            last = node;
            e = hipStreamBeginCapture(st, hipStreamCaptureModeThreadLocal);
            capturing = e == hipSuccess;
        }
        return e;
    }
    hipError_t finish(hipGraph_t *out) {
        hipError_t e = close_segment();
        if (e == hipSuccess) {
            *out = g;
            g = nullptr;
        }
        return e;
    }
    ~ChunkBuilder() {
        if (capturing) {
            hipGraph_t seg = nullptr;
            (void)hipStreamEndCapture(st, &seg);
            if (seg) (void)hipGraphDestroy(seg);
        }
        if (g) (void)hipGraphDestroy(g);
    }
};

// Iterations of a chunk whose passes are bracketed by events (profile = N: every N-th).
int profiled_iters(const hprlp_handle *h) {
    const int L = (int)h->opt.check_every, N = h->opt.profile;
    return (N > 0 && !h->no_graph_events) ? (L + N - 1) / N : 0;
}

// Record one chunk of check_every iterations on the library stream: first iteration (keep)
// + its check sums, plain iterations, last iteration (keep) + check sums, the decisions of
// every instance, the restart copies, and the iteration counter advance.  With profile = N,
// the passes of every N-th iteration are bracketed by events 3q, 3q+1 (after the column
// pass) and 3q+2 (after the row pass) of the event pool, marked through `cb`.
int record_chunk(hprlp_handle *h, int prec, ChunkBuilder *cb) {
    const int L = (int)h->opt.check_every;
    const int N = cb && profiled_iters(h) > 0 ? h->opt.profile : 0;
    const void *vs = pass_set(h, prec);
    const int cp = check_prec(prec);
    const IterScalars unused{};  // batched passes read their scalars from device memory
    hipError_t e = hipSuccess;
    for (int i = 0; i < L && e == hipSuccess; ++i) {
        const bool keep = (i == 0 || i == L - 1);
        const bool samp = N > 0 && i % N == 0;
        const size_t e0 = samp ? (size_t)(3 * (i / N)) : 0;
        const BatchArgs ba = batch_args(h, i);
        if (samp) e = cb->mark(h->ev_pool[e0]);
        if (e == hipSuccess) e = launch_col_pass(prec, keep, h->T, vs, unused, h->st, nullptr, &ba);
        if (e == hipSuccess && samp) e = cb->mark(h->ev_pool[e0 + 1]);
        if (e == hipSuccess) e = launch_row_pass(prec, keep, h->A, vs, unused, h->st, nullptr, &ba);
        if (e == hipSuccess && samp) e = cb->mark(h->ev_pool[e0 + 2]);
        if (e == hipSuccess && keep) {
            double *res = i == 0 ? h->bd.res_first : h->bd.res_chk;
            e = launch_check_row(cp, h->A, pass_set(h, cp), h->chk, h->v64.bd, 0, h->partsA,
                                 res, h->st, &ba, &h->segA, 2 * kNQ);
            if (e == hipSuccess)
                e = launch_check_col(cp, h->T, pass_set(h, cp), h->chk, h->v64.cd, h->v64.sc,
                                     h->partsT, res + kNQ, h->st, &ba, &h->segT, 2 * kNQ);
        }
    }
    if (e != hipSuccess) return fail(h, HPRLP_EHIP, std::string("chunk launch: ") + hipGetErrorString(e));
    const hprlp_options &o = h->opt;
    DecideArgs d;
    d.n_inst = h->n_inst; d.chunk = L; d.max_iter = o.max_iter;
    d.tol = o.tol; d.alpha1 = o.alpha1; d.alpha2 = o.alpha2; d.alpha3 = o.alpha3;
    d.tol_switch = o.tol_switch; d.use_restart = o.use_restart; d.sigma_update = o.sigma_update;
    d.res_first = h->bd.res_first; d.res_chk = h->bd.res_chk; d.cst = h->bd.cst;
    d.sigma = h->bd.sigma; d.lam = h->bd.lam; d.merit0 = h->bd.merit0;
    d.merit_prev = h->bd.merit_prev; d.kstart = h->bd.kstart; d.kbase = h->bd.kbase;
    d.iters_done = h->bd.iters_done; d.restarts = h->bd.restarts; d.nchecks = h->bd.nchecks;
    d.active = h->bd.active; d.status = h->bd.status; d.restart_flag = h->bd.restart_flag;
    d.last = h->bd.last; d.trace = h->bd.trace; d.summary = h->bd.summary;
    e = launch_decide(d, h->st);
    if (e == hipSuccess && prec == 1) {  // FP32 phase: move the anchors, renew its data
        e = launch_reanchor_batched(h->vdisp, h->bd.row_off, h->bd.col_off, h->bd.restart_flag,
                                    h->n_inst, h->st);
        if (e == hipSuccess) e = launch_anchor(h->A, h->T, h->vdisp, h->st);
    } else if (e == hipSuccess) {
        e = launch_restart_batched(false, vs, h->bd.row_off, h->bd.col_off, h->bd.restart_flag,
                                   h->n_inst, h->st);
    }
    if (e == hipSuccess) e = launch_advance(h->bd.kbase, L, h->st);
    if (e != hipSuccess) return fail(h, HPRLP_EHIP, std::string("chunk launch: ") + hipGetErrorString(e));
    return HPRLP_OK;
}

// The chunk graph of one precision phase, captured on first use and kept with the handle.
int get_graph(hprlp_handle *h, int prec, hipGraphExec_t *out) {
    if (!h->graphs[prec]) {
        hipGraph_t g = nullptr;
        if (profiled_iters(h) > 0) {
            // the events of the event nodes exist before the capture starts
            for (int q = 0; q < 3 * profiled_iters(h); ++q)
                if (!pool_event(h, (size_t)q)) return fail(h, HPRLP_EHIP, "hipEventCreate failed");
            ChunkBuilder cb{h->st};
            hipError_t e = cb.start();
            int rc = e == hipSuccess ? record_chunk(h, prec, &cb) : HPRLP_OK;
            if (e == hipSuccess && rc == HPRLP_OK) e = cb.finish(&g);
            if (e != hipSuccess || rc != HPRLP_OK) {  // event nodes refused: a graph without
                h->graph_event_error = rc ? h->err : std::string(hipGetErrorString(e));
                (void)hipGetLastError();
                h->no_graph_events = true;
                if (h->opt.verbose)
                    std::fprintf(stderr, "hprlp: chunk graph without event nodes (%s)\n",
                                 h->graph_event_error.c_str());
                g = nullptr;
            }
        }
        if (!g) {
            HIPCHK(h, hipStreamBeginCapture(h->st, hipStreamCaptureModeThreadLocal));
            const int rc = record_chunk(h, prec, nullptr);
            const hipError_t e = hipStreamEndCapture(h->st, &g);
            if (rc || e != hipSuccess) {
                if (g) (void)hipGraphDestroy(g);
                if (rc) return rc;
                return fail(h, HPRLP_EHIP, std::string("hipStreamEndCapture: ") + hipGetErrorString(e));
            }
        }
        hipGraphExec_t ex = nullptr;
        const hipError_t e2 = hipGraphInstantiate(&ex, g, nullptr, nullptr, 0);
        (void)hipGraphDestroy(g);
        if (e2 != hipSuccess) return fail(h, HPRLP_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e2));
        h->graphs[prec] = ex;
    }
    *out = h->graphs[prec];
    return HPRLP_OK;
}

// Start of a batched solve: every instance at the origin with sigma = sigma0, k = 0, and
// lambda per instance from the caller, lambda_override or the power method (Section 4.1).
int batch_begin(hprlp_handle *h, int *status) {
    const hprlp_options &o = h->opt;
    const int ni = h->n_inst;
    if (h->user_st) HIPCHK(h, hipStreamSynchronize(h->user_st));
    BatchRun &br = h->br;
    br = BatchRun{};
    br.t_start = now_ms();
    h->solved = false;  // outputs of an earlier solve are no longer the handle's
    h->stats = hprlp_stats_t{};
    h->inst_stats.clear();
    h->prec = h->f32phase ? 1 : (h->mixed ? 2 : 0);
    h->n_compactions = 0;
    int rc;
    if (h->compacted && (rc = set_schedules(h, {}))) return rc;
    if ((rc = init_batch_state(h, o.sigma0, 0.0))) return rc;
    br.lam.assign((size_t)ni, o.lambda_override);
    if (!h->lam_given.empty()) br.lam = h->lam_given;
    else if (!(o.lambda_override > 0) && (rc = power_method(h, br.lam, &br.piters))) return rc;
    for (int b = 0; b < ni; ++b)
        if (!(br.lam[b] > 0.0) || !std::isfinite(br.lam[b])) {
            h->stats.status = HPRLP_NUMERICAL;
            if (status) *status = HPRLP_NUMERICAL;
            return fail(h, HPRLP_OK, "power method gave lambda <= 0 for instance " + std::to_string(b));
        }
    if ((rc = upload(h, h->bd.lam, br.lam.data(), br.lam.size()))) return rc;
    br.t_power = now_ms() - br.t_start;
    if ((rc = zero_state(h))) return rc;
    br.prev_active = (double)ni;
    br.begun = true;
    return HPRLP_OK;
}

// Run up to max_chunks chunks (< 0: until every instance has stopped or a limit of the
// options is hit).  Each chunk is one launch of the captured graph and one 32-byte
// read-back of the summary; stopped instances are dropped from the schedules as they
// accumulate, and a MIXED batch switches to FP64 per reading 22 of the design.
int batch_run(hprlp_handle *h, long long max_chunks) {
    const hprlp_options &o = h->opt;
    const int ni = h->n_inst;
    BatchRun &br = h->br;
    int rc;
    for (long long c = 0; (max_chunks < 0 || c < max_chunks) && !br.done; ++c) {
        hipGraphExec_t ex;
        if ((rc = get_graph(h, h->prec, &ex))) return rc;
        HIPCHK(h, hipGraphLaunch(ex, h->st));
        if ((rc = download(h, h->pinned, h->bd.summary, 4))) return rc;
        const double t_chunk = now_ms() - br.t_start;
        const double n_active = h->pinned[0], max_kkt = h->pinned[1], n_above = h->pinned[2];
        br.k = (long long)h->pinned[3];
        br.chunk_end.push_back({br.k, t_chunk});
        if (h->prec == 1) br.iters_fp32 = br.k;
        for (int q = 0; q < profiled_iters(h); ++q) {  // the graph's event nodes of this chunk
            float a = 0.f, b2 = 0.f;
            HIPCHK(h, hipEventElapsedTime(&a, h->ev_pool[3 * q], h->ev_pool[3 * q + 1]));
            HIPCHK(h, hipEventElapsedTime(&b2, h->ev_pool[3 * q + 1], h->ev_pool[3 * q + 2]));
            br.prof_ms[0] += a;
            br.prof_ms[1] += b2;
            br.prof_n[0] += 1;
            br.prof_n[1] += 1;
        }
        if (o.verbose)
            std::fprintf(stderr, "hprlp batch k=%lld active=%.0f max_kkt=%.2e scheduled_nnz=%lld\n",
                         br.k, n_active, max_kkt, (long long)h->sched_nnz);
        if (n_active == 0) {
            br.prev_active = 0.0;
            br.done = true;
            break;
        }
        if (n_active < br.prev_active) {
            // drop the stopped instances from the schedules once they hold an eighth of the
            // scheduled nonzeros (their work items still stream their nonzeros; only the
            // writes are skipped)
            std::vector<int> act((size_t)ni);
            if ((rc = download(h, act.data(), h->bd.active, act.size()))) return rc;
            int64_t live = 0;
            for (int b = 0; b < ni; ++b)
                if (act[b]) live += h->inst_nnz[b];
            if (live <= (h->sched_nnz * 7) / 8) {
                if ((rc = set_schedules(h, act))) return rc;
                h->n_compactions++;
            }
            br.prev_active = n_active;
        }
        if (br.k >= o.max_iter) {
            br.st_all = HPRLP_ITER_LIMIT;
            br.done = true;
            break;
        }
        if (o.time_limit > 0 && t_chunk / 1000.0 >= o.time_limit) {
            br.st_all = HPRLP_TIME_LIMIT;
            br.done = true;
            break;
        }
        if (h->prec == 1) {
            // as for one LP, on the largest rel. KKT over the instances still iterating
            bool sw = n_above == 0;
            br.kkt_hist.push_back(max_kkt);
            const size_t S = (size_t)o.stall_checks, H = br.kkt_hist.size();
            if (!sw && S > 0 && H > S) {
                const double before = *std::min_element(br.kkt_hist.begin(), br.kkt_hist.end() - S);
                const double recent = *std::min_element(br.kkt_hist.end() - S, br.kkt_hist.end());
                sw = recent > o.stall_ratio * before;
            }
            if (sw && (rc = promote(h))) return rc;
        }
    }
    HIPCHK(h, hipStreamSynchronize(h->st));
    return HPRLP_OK;
}

// Per-instance and summed statistics of the batch as it stands.  An instance that stopped
// reports the time from the start of the solve to the end of the chunk whose check stopped
// it (t_solve_ms); one still iterating reports the time so far.
int batch_stats(hprlp_handle *h, int *status) {
    const hprlp_options &o = h->opt;
    const int ni = h->n_inst;
    BatchRun &br = h->br;
    const double t_end = br.chunk_end.empty() ? br.t_power : br.chunk_end.back().second;
    std::vector<int> ist((size_t)ni);
    std::vector<long long> idone((size_t)ni), irest((size_t)ni), inch((size_t)ni);
    std::vector<double> isig((size_t)ni), ilast((size_t)ni * 6), cst((size_t)ni * 8);
    int rc;
    if ((rc = download(h, ist.data(), h->bd.status, ist.size())) ||
        (rc = download(h, idone.data(), h->bd.iters_done, idone.size())) ||
        (rc = download(h, irest.data(), h->bd.restarts, irest.size())) ||
        (rc = download(h, inch.data(), h->bd.nchecks, inch.size())) ||
        (rc = download(h, isig.data(), h->bd.sigma, isig.size())) ||
        (rc = download(h, ilast.data(), h->bd.last, ilast.size())) ||
        (rc = download(h, cst.data(), h->bd.cst, cst.size())))
        return rc;
    h->inst_stats.assign((size_t)ni, hprlp_stats_t{});
    hprlp_stats_t s{};
    int worst = HPRLP_OPTIMAL;
    for (int b = 0; b < ni; ++b) {
        hprlp_stats_t &q = h->inst_stats[b];
        q.status = ist[b] ? ist[b] : br.st_all;
        q.iters = ist[b] ? idone[b] : br.k;
        q.restarts = irest[b];
        q.sigma = isig[b];
        q.lambda = br.lam[b];
        q.power_iters = br.piters;
        q.rel_p = ilast[b * 6 + 0]; q.rel_d = ilast[b * 6 + 1]; q.rel_gap = ilast[b * 6 + 2];
        q.pobj = ilast[b * 6 + 3]; q.dobj = ilast[b * 6 + 4];
        q.beta_b = cst[(size_t)b * 8 + 0];
        q.beta_c = cst[(size_t)b * 8 + 1];
        q.t_solve_ms = t_end;
        if (ist[b])
            for (const auto &ce : br.chunk_end)
                if (ce.first == idone[b]) {
                    q.t_solve_ms = ce.second;
                    break;
                }
        q.t_power_ms = br.t_power;
        q.n_checks = inch[b];
        if (q.status != HPRLP_OPTIMAL && worst == HPRLP_OPTIMAL) worst = q.status;
        s.restarts += q.restarts;
        s.rel_p = std::max(s.rel_p, q.rel_p);
        s.rel_d = std::max(s.rel_d, q.rel_d);
        s.rel_gap = std::max(s.rel_gap, q.rel_gap);
        s.pobj += q.pobj;
        s.dobj += q.dobj;
    }
    s.iters = br.k;
    s.iters_fp32 = h->f32phase ? br.iters_fp32 : 0;
    s.status = worst;
    s.power_iters = br.piters;
    s.t_power_ms = br.t_power;
    s.t_solve_ms = t_end;
    s.bytes_per_iter = bytes_per_iter(h);
    s.col_pass_ms = br.prof_ms[0];
    s.row_pass_ms = br.prof_ms[1];
    s.col_pass_launches = br.prof_n[0];
    s.row_pass_launches = br.prof_n[1];
    s.n_checks = br.k / o.check_every;
    s.n_compactions = h->n_compactions;
    s.t_setup_ms = h->t_setup_ms;
    s.t_prep_ms = h->t_prep_ms;
    s.t_tune_ms = h->t_tune_ms;
    h->stats = s;
    if (status) *status = worst;
    return HPRLP_OK;
}

int solve_batched(hprlp_handle *h, double *x, double *y, double *z, int *status) {
    int rc;
    if ((rc = batch_begin(h, status))) return rc;
    if (!h->br.begun) return HPRLP_OK;  // lambda <= 0: status NUMERICAL already reported
    if ((rc = batch_run(h, -1))) return rc;
    if ((rc = write_outputs(h, x, y, z))) return rc;
    h->solved = true;
    return batch_stats(h, status);
}

}  // namespace

extern "C" int hprlp_solve(hprlp_handle *h, double *x, double *y, double *z, int *status) {
    if (!h) return fail(nullptr, HPRLP_EINVAL, "null handle");
    return h->batched ? solve_batched(h, x, y, z, status) : solve_single(h, x, y, z, status);
}

extern "C" int hprlp_stats(const hprlp_handle *h, hprlp_stats_t *out) {
    if (!h || !out) return fail(const_cast<hprlp_handle *>(h), HPRLP_EINVAL, "null argument");
    *out = h->stats;
    return HPRLP_OK;
}

extern "C" int hprlp_stats_instance(const hprlp_handle *hc, int32_t i, hprlp_stats_t *out) {
    hprlp_handle *h = const_cast<hprlp_handle *>(hc);
    if (!h || !out) return fail(h, HPRLP_EINVAL, "null argument");
    if (i < 0 || i >= h->n_inst) return fail(h, HPRLP_EINVAL, "instance index out of range");
    if (!h->batched) {
        *out = h->stats;
        return HPRLP_OK;
    }
    if (h->inst_stats.empty()) return fail(h, HPRLP_ESTATE, "no solve has run yet");
    *out = h->inst_stats[i];
    return HPRLP_OK;
}

extern "C" int hprlp_get_iterate(const hprlp_handle *hc, int which, double *out) {
    hprlp_handle *h = const_cast<hprlp_handle *>(hc);
    if (!h || !out) return fail(h, HPRLP_EINVAL, "null argument");
    if (which == HPRLP_DROW || which == HPRLP_DCOL) {
        const std::vector<double> &d = which == HPRLP_DROW ? h->dr : h->dc;
        HIPCHK(h, hipMemcpy(out, d.data(), d.size() * sizeof(double), hipMemcpyDefault));
        return HPRLP_OK;
    }
    if (!h->solved) return fail(h, HPRLP_ESTATE, "no solve has run yet");
    if (h->batched && which == HPRLP_XCUR)
        return fail(h, HPRLP_EINVAL, "XCUR needs one inner counter; a batch has one per instance");
    const bool disp = h->prec == 1;  // FP32 phase: current iterate = anchor + displacement
    double *tmp = h->outv;
    hipError_t e = hipSuccess;
    long long len = 0;
    switch (which) {  // w_bar is FP64 in every phase
    case HPRLP_XBAR:
        e = launch_scale_out(tmp, h->v64.xbar, false, h->ux, 0, h->cperm, h->n, h->st);
        len = h->n;
        break;
    case HPRLP_YBAR:
        e = launch_scale_out(tmp, h->v64.ybar, false, h->uy, 0, nullptr, h->m, h->st);
        len = h->m;
        break;
    case HPRLP_ZBAR:
        e = launch_scale_out(tmp, h->v64.zint, false, h->chk.co, 0, h->cperm, h->n, h->st);
        len = h->n;
        break;
    case HPRLP_XCUR: {
        IterScalars s;
        fill_scalars(h, s);
        if (disp)
            e = launch_anchor_out(tmp, h->v64.x0, h->vdisp.dxrel ? h->vdisp.dxrel : h->vdisp.dxh,
                                  s.hx1, h->ux, h->cperm, h->n, h->st);
        else
            e = launch_xcur_out(tmp, h->v64.x0, h->v64.xrel ? h->v64.xrel : h->v64.xhat, false,
                                s.hx0, s.hx1, h->ux, 0, h->cperm, h->n, h->st);
        len = h->n;
        break;
    }
    case HPRLP_YCUR:
        if (disp)
            e = launch_anchor_out(tmp, h->v64.y0, h->vdisp.dy, 1.0, h->uy, nullptr, h->m, h->st);
        else
            e = launch_scale_out(tmp, h->v64.y, false, h->uy, 0, nullptr, h->m, h->st);
        len = h->m;
        break;
    default:
        return fail(h, HPRLP_EINVAL, "unknown iterate");
    }
    if (e != hipSuccess) return fail(h, HPRLP_EHIP, hipGetErrorString(e));
    return copy_out(h, out, tmp, len);
}

extern "C" int hprlp_get_trace(const hprlp_handle *hc, double *out, long long cap,
                               long long *n_rows) {
    hprlp_handle *h = const_cast<hprlp_handle *>(hc);
    if (!h || !n_rows) return fail(h, HPRLP_EINVAL, "null argument");
    *n_rows = (long long)h->trace.size();
    if (out)
        for (long long i = 0; i < std::min<long long>(cap, *n_rows); ++i)
            std::memcpy(out + i * TR_NCOL, h->trace[i].data(), TR_NCOL * sizeof(double));
    return HPRLP_OK;
}

extern "C" int hprlp_get_trace_instance(const hprlp_handle *hc, int32_t i, double *out,
                                        long long cap, long long *n_rows) {
    hprlp_handle *h = const_cast<hprlp_handle *>(hc);
    if (!h || !n_rows) return fail(h, HPRLP_EINVAL, "null argument");
    if (!h->batched) return fail(h, HPRLP_EINVAL, "not a batched handle");
    if (i < 0 || i >= h->n_inst) return fail(h, HPRLP_EINVAL, "instance index out of range");
    if (!h->solved) return fail(h, HPRLP_ESTATE, "no solve has run yet");
    long long nc = 0;
    int rc = download(h, &nc, h->bd.nchecks + i, 1);
    if (rc) return rc;
    *n_rows = std::min<long long>(nc, kTraceRows);
    const long long k = std::min<long long>(cap, *n_rows);
    if (out && k > 0)
        rc = download(h, out, h->bd.trace + (size_t)i * kTraceRows * kTraceCols,
                      (size_t)k * kTraceCols);
    return rc;
}

extern "C" int hprlp_get_schedule(const hprlp_handle *hc, int matrix, int32_t *params,
                                  int64_t *counts, double *tuned_ms) {
    hprlp_handle *h = const_cast<hprlp_handle *>(hc);
    if (!h || (matrix != 0 && matrix != 1)) return fail(h, HPRLP_EINVAL, "bad argument");
    const ScheduleParams &p = matrix == 0 ? h->spA : h->spT;
    const Schedule &S = (matrix == 0 ? h->A : h->T).host;
    if (params) {
        params[0] = p.tile_nnz; params[1] = p.tile_rows; params[2] = p.short_max;
        params[3] = p.split_len; params[4] = p.chunk_nnz;
    }
    if (counts) {
        counts[0] = (int64_t)S.items.size(); counts[1] = S.n_tiles; counts[2] = S.n_rowitems;
        counts[3] = S.n_chunks;
        counts[4] = (matrix == 0 ? h->A : h->T).sorted ? 1 : 0;
        counts[5] = S.n_bundle_items;
    }
    if (tuned_ms) *tuned_ms = h->tuned_ms[matrix];
    return HPRLP_OK;
}

extern "C" int hprlp_begin(hprlp_handle *h) {
    if (!h) return fail(h, HPRLP_EINVAL, "null handle");
    int st = 0, rc;
    if (h->batched) {
        if ((rc = batch_begin(h, &st))) return rc;
        if (!h->br.begun) return HPRLP_OK;  // NUMERICAL in the stats; hprlp_step refuses
        h->solved = true;
        return batch_stats(h, nullptr);
    }
    HIPCHK(h, hipStreamSynchronize(h->st));
    const double t0 = now_ms();
    int piters = 0;
    if ((rc = single_begin(h, &st, &piters))) return rc;
    if (h->stats.status == HPRLP_NUMERICAL) return HPRLP_OK;
    HIPCHK(h, hipStreamSynchronize(h->st));
    h->solved = true;
    h->stats.power_iters = piters;
    h->stats.lambda = h->opt.t1_zero ? 0.0 : h->lambda;
    h->stats.sigma = h->sigma;
    h->stats.t_power_ms = now_ms() - t0;
    h->stats.t_setup_ms = h->t_setup_ms;
    h->stats.t_prep_ms = h->t_prep_ms;
    h->stats.t_tune_ms = h->t_tune_ms;
    return HPRLP_OK;
}

extern "C" int hprlp_step(hprlp_handle *h, int iters) {
    if (!h || iters < 0) return fail(h, HPRLP_EINVAL, "bad argument");
    if (!h->solved) return fail(h, HPRLP_ESTATE, "call after hprlp_begin or a solve");
    if (h->batched) {
        const long long ce = h->opt.check_every;
        if (iters % ce != 0)
            return fail(h, HPRLP_EINVAL, "a batched step runs whole chunks: iters must be a "
                                         "multiple of check_every");
        if (!h->br.begun) return fail(h, HPRLP_ESTATE, "call after hprlp_begin or a solve");
        // nothing left to run once every instance has stopped or a limit is reached
        const hprlp_options &o = h->opt;
        const bool timed_out =
            o.time_limit > 0 && (now_ms() - h->br.t_start) / 1000.0 >= o.time_limit;
        if (h->br.prev_active == 0.0 || h->br.k >= o.max_iter || timed_out) return HPRLP_OK;
        h->br.done = false;
        int rc = batch_run(h, iters / ce);
        if (rc) return rc;
        return batch_stats(h, nullptr);
    }
    size_t ev = 0;
    for (int i = 0; i < iters; ++i) {
        const int rc = run_iteration(h, false, nullptr, &ev);
        if (rc) return rc;
    }
    HIPCHK(h, hipStreamSynchronize(h->st));
    h->stats.iters = h->k;
    return HPRLP_OK;
}

extern "C" int hprlp_time_passes(hprlp_handle *h, int reps, double *col_ms, double *row_ms) {
    if (!h || reps < 1) return fail(h, HPRLP_EINVAL, "bad argument");
    if (!h->solved) return fail(h, HPRLP_ESTATE, "call after a solve");
    IterScalars s;
    fill_scalars(h, s);
    const void *vs = cur_set(h);
    const BatchArgs ba = batch_args(h, 0);
    const BatchArgs *pba = h->batched ? &ba : nullptr;
    if (h->batched) {  // time every instance's work, whatever the last solve left active
        std::vector<int> ones((size_t)h->n_inst, 1);
        int rc = upload(h, h->bd.active, ones.data(), ones.size());
        if (rc) return rc;
        if (h->compacted && (rc = set_schedules(h, {}))) return rc;
    }
    hipEvent_t e[4];
    for (int i = 0; i < 4; ++i) {
        e[i] = pool_event(h, i);
        if (!e[i]) return fail(h, HPRLP_EHIP, "hipEventCreate failed");
    }
    HIPCHK(h, hipEventRecord(e[0], h->st));
    for (int i = 0; i < reps; ++i) {
        hipError_t r = launch_col_pass(h->prec, false, h->T, vs, s, h->st, nullptr, pba);
        if (r != hipSuccess) return fail(h, HPRLP_EHIP, hipGetErrorString(r));
    }
    HIPCHK(h, hipEventRecord(e[1], h->st));
    HIPCHK(h, hipEventRecord(e[2], h->st));
    for (int i = 0; i < reps; ++i) {
        hipError_t r = h->batched ? launch_row_pass(h->prec, false, h->A, vs, s, h->st, nullptr, pba)
                                  : row_step(h, false, s, vs, nullptr);
        if (r != hipSuccess) return fail(h, HPRLP_EHIP, hipGetErrorString(r));
    }
    HIPCHK(h, hipEventRecord(e[3], h->st));
    HIPCHK(h, hipEventSynchronize(e[3]));
    float a = 0, b = 0;
    HIPCHK(h, hipEventElapsedTime(&a, e[0], e[1]));
    HIPCHK(h, hipEventElapsedTime(&b, e[2], e[3]));
    if (col_ms) *col_ms = a / reps;
    if (row_ms) *row_ms = b / reps;
    return HPRLP_OK;
}

extern "C" const char *hprlp_last_error(const hprlp_handle *h) {
    return h ? h->err.c_str() : g_create_error.c_str();
}

extern "C" void hprlp_destroy(hprlp_handle *h) {
    if (!h) return;
    for (hipGraphExec_t g : h->graphs)
        if (g) (void)hipGraphExecDestroy(g);
    for (hipEvent_t e : h->ev_pool) (void)hipEventDestroy(e);
    if (h->pinned) {
        if (h->noalloc) delete[] h->pinned;
        else (void)hipHostFree(h->pinned);
    }
    if (h->noalloc) release_scratch(h);
    if (h->own_stream && h->st) (void)hipStreamDestroy(h->st);
    if (h->cap_st) (void)hipStreamDestroy(h->cap_st);
    delete h;
}
