// HIP kernels of the HPR-LP iteration for gfx950 (CDNA4).
//
// The two sparse products of one iteration (Section 3.3 of the paper: eqs. update-z,
// update-x and update-y-2) are each ONE binned CSR SpMV launch whose epilogue applies the
// whole vector update of that half-step: projection onto the box C or the cone D,
// reflection w_hat = 2 w_bar - w, and the Halpern averaging of Algorithm 2.  The stored
// transpose turns A^T y into a row-wise product, so no pass needs atomics and every sum is
// taken in a fixed order (bit-reproducible runs).
//
// Work items (one 256-thread workgroup each, see Schedule):
//   TILE   a run of consecutive short rows holding <= tile_nnz nonzeros.  Phase 1 streams the
//          tile's nonzeros with fully coalesced loads and stages the products in LDS;
//          phase 2 sums each row from LDS with a group of G lanes (G = power of two sized to
//          the tile's rows, reduced by cross-lane shuffles); phase 3 runs the epilogue with
//          one thread per row, so vector loads/stores of the epilogue are coalesced too.
//   ROW    one long row summed by the whole workgroup (wavefront shuffles + LDS).
//   CHUNK  a slice of a very long row; its partial sum goes to a slot and a second small
//          kernel adds the slots of each split row in index order and runs the epilogue.
// The host lays the items out XCD-aware: workgroup b runs on XCD b % 8, and each item class
// is interleaved so that every XCD walks a contiguous range of it (rows that share gathered
// cache lines stay on one XCD's L2) while all XCDs see the same mix of heavy and light work.
// Check passes (every check_every iterations) reuse the same kernel with epilogues that
// produce per-workgroup partial sums of the termination / restart / sigma quantities,
// reduced in a fixed order (one workgroup for a single LP, one per instance for a batch).
//
// Batched solves (many LPs packed block-diagonally) run the same passes; each work item
// belongs to one instance, and its scalars (sigma, lambda, the Halpern counter, the first
// inequality row, whether it still iterates) come from per-instance device arrays, so a
// whole chunk of iterations can be captured once in a hipGraph.
#include <algorithm>

#include "hprlp_internal.h"

namespace hprlp {
namespace {

struct D2 {
    double a, b;
};
__device__ __forceinline__ D2 operator+(D2 x, D2 y) { return D2{x.a + y.a, x.b + y.b}; }

template <class S> __device__ __forceinline__ S szero();
template <> __device__ __forceinline__ float szero<float>() { return 0.f; }
template <> __device__ __forceinline__ double szero<double>() { return 0.0; }
template <> __device__ __forceinline__ D2 szero<D2>() { return D2{0.0, 0.0}; }

__device__ __forceinline__ float xshfl(float v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ double xshfl(double v, int m) { return __shfl_xor(v, m, 64); }
__device__ __forceinline__ D2 xshfl(D2 v, int m) {
    return D2{__shfl_xor(v.a, m, 64), __shfl_xor(v.b, m, 64)};
}

template <class S> __device__ __forceinline__ S wave_sum(S v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v = v + xshfl(v, off);
    return v;
}

// Sum over the 256 threads of the workgroup; the result is valid in thread 0.
template <class S> __device__ __forceinline__ S block_sum(S v, S *red) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    S t = szero<S>();
    if (threadIdx.x == 0) t = ((red[0] + red[1]) + red[2]) + red[3];
    return t;
}

template <class V> __device__ __forceinline__ V vmin(V a, V b) { return a < b ? a : b; }
template <class V> __device__ __forceinline__ V vmax(V a, V b) { return a > b ? a : b; }
// Box projection with +-inf bounds (fmin/fmax semantics: a NaN bound is never produced).
template <class V> __device__ __forceinline__ V clampv(V v, V lo, V hi) {
    return vmin(vmax(v, lo), hi);
}

template <class M, class V> struct AccT { using type = double; };
template <> struct AccT<float, float> { using type = float; };

// Scalars one work item needs: from kernel arguments (single LP) or from the per-instance
// arrays of a batched solve.  Halpern weights of Algorithm 2 at inner counter t:
// x^{r,t} = x0/(t+1) + t/(t+1) x_hat, y^{r,t+1} = y0/(t+2) + (t+1)/(t+2) y_hat.
struct PassCtx {
    double sigma, lam_sigma, hx0, hx1, hy0, hy1, inv_norm, rho;
    long long m1_end;
    int active;
};

__device__ __forceinline__ PassCtx ctx_single(const IterScalars &s, const double *inv_norm) {
    PassCtx c;
    c.sigma = s.sigma;
    c.lam_sigma = s.lam_sigma;
    c.hx0 = s.hx0; c.hx1 = s.hx1; c.hy0 = s.hy0; c.hy1 = s.hy1;
    c.inv_norm = inv_norm ? *inv_norm : 1.0;
    c.m1_end = s.m1;
    c.active = 1;
    c.rho = s.rho;
    return c;
}

__device__ __forceinline__ PassCtx ctx_batch(const BatchArgs &b, int inst) {
    PassCtx c;
    c.active = b.active[inst];
    const double sg = b.sigma[inst];
    c.sigma = sg;
    c.lam_sigma = b.lam[inst] * sg;
    const double t = (double)((*b.kbase + b.iter_off) - b.kstart[inst]);
    if (b.halpern) {
        c.hx0 = 1.0 / (t + 1.0);
        c.hx1 = t / (t + 1.0);
        c.hy0 = 1.0 / (t + 2.0);
        c.hy1 = (t + 1.0) / (t + 2.0);
    } else {
        c.hx0 = 0.0; c.hx1 = 1.0; c.hy0 = 0.0; c.hy1 = 1.0;
    }
    c.m1_end = b.m1_end[inst];
    c.inv_norm = b.inv_norm ? b.inv_norm[inst] : 1.0;
    c.rho = b.rho;
    return c;
}

// ------------------------------------------------------------------------- the SpMV kernel
//
// Op interface (one per pass kind):
//   PassCtx begin(inst)       scalars of the work item's instance
//   Raw raw(p)                nonzero p: column index and value, loaded with a streaming hint
//   Sum prod(const Raw&)      gather of the input vector(s) and product
//   Pre load(row)             epilogue operands of one row (prefetched when PREFETCH)
//   void apply(row, sum, pre, ctx, q)   the fused epilogue; q accumulates check terms
// Loads are issued in batches of kEPT per thread (all indices/values first, then all
// gathers) so each workgroup pays two memory latencies per batch instead of one per element.

constexpr int kEPT = 8;   // nonzeros per thread per batch (tile_nnz <= kWG * kEPT)
constexpr int kRPT = 4;   // rows per thread in the tile epilogue (tile_rows <= kWG * kRPT)
// Epilogue operands are prefetched (issued before the nonzero stream) for the first kPRE rows
// of each thread only: tiles rarely have more than kWG rows, and holding kRPT rows of operands
// through the SpMV phases would cost the registers that keep more workgroups resident.
constexpr int kPRE = 1;

template <class M> struct RawT {
    int j;
    M a;
};
template <class M>
__device__ __forceinline__ RawT<M> load_raw(const int *__restrict__ ci, const M *__restrict__ va,
                                            int p) {
    return RawT<M>{__builtin_nontemporal_load(ci + p), __builtin_nontemporal_load(va + p)};
}

struct NoPre {};

// Epilogue vector access of the x-step: with FP64 vectors the five operand reads and the
// x_hat write bypass cache retention (measured inside solves: column pass 5-6% faster on
// zipf1m and transport10m, as the gathered y keeps more of L2); with FP32 vectors plain
// accesses are faster (16% on the FP32 phase of transport10m).
template <class V> __device__ __forceinline__ V ep_load(const V *p) {
    if constexpr (sizeof(V) == 8) return __builtin_nontemporal_load(p);
    else return *p;
}
template <class V> __device__ __forceinline__ void ep_store(V *p, V v) {
    if constexpr (sizeof(V) == 8) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Sum of op.prod over nonzeros [b, e) by the whole workgroup (e > b).  The batch is
// branch-free: out-of-range lanes re-load the last nonzero (a cache hit) and contribute zero
// through a select, so all kEPT index/value loads and then all kEPT gathers are in flight
// together.
template <class Op>
__device__ __forceinline__ typename Op::Sum row_sum(const Op &op, int b, int e, int tid) {
    using S = typename Op::Sum;
    S s = szero<S>();
    for (int base = b; base < e; base += kWG * kEPT) {
        typename Op::Raw raw[kEPT];
#pragma unroll
        for (int u = 0; u < kEPT; ++u) raw[u] = op.raw(min(base + tid + u * kWG, e - 1));
        S v[kEPT];
#pragma unroll
        for (int u = 0; u < kEPT; ++u) v[u] = op.prod(raw[u]);
#pragma unroll
        for (int u = 0; u < kEPT; ++u) s = s + (base + tid + u * kWG < e ? v[u] : szero<S>());
    }
    return s;
}

// POS: the tiles hold their nonzeros in column order and pos[p] is the row-order offset
// (inside its tile) of the nonzero stored at p; each product is staged at that offset, so
// the sums below see the row order either way.  (A template parameter, so the row-order
// kernel keeps its registers.)
template <class Op, bool POS>
__global__ __launch_bounds__(kWG) void k_pass(const int4 *__restrict__ items,
                                              const int *__restrict__ rp, Op op,
                                              typename Op::Sum *__restrict__ split_part,
                                              double *__restrict__ parts, int tile_cap,
                                              int rows_cap,
                                              const unsigned short *__restrict__ pos) {
    using S = typename Op::Sum;
    using Pre = typename Op::Pre;
    constexpr int NQ = Op::NQ > 0 ? Op::NQ : 1;
    extern __shared__ __align__(16) unsigned char smem[];
    __shared__ S red[4];
    __shared__ double redq[4];
    const int4 it = items[blockIdx.x];
    const int kind = it.w & kKindMask;
    const int tid = threadIdx.x;
    double q[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) q[j] = 0.0;

    // The loads of a work item are issued before its instance's active flag is known (a
    // batched solve's scalars come from memory): only the epilogue writes wait for it.
    // Stopped instances are dropped from the schedules by the host as they accumulate.
    if (kind == IT_TILE) {
        const int r0 = it.x, P0 = it.y, inst = it.z;
        const PassCtx ctx = op.begin(inst);
        {
            S *prod = reinterpret_cast<S *>(smem);
            S *rsum = prod + tile_cap;
            int *rpl = reinterpret_cast<int *>(rsum + rows_cap);
            const int nrows = it.w >> 15, cnt = (it.w >> kKindBits) & 4095;
            const int r1 = r0 + nrows;
            Pre pre[kPRE];
            if constexpr (Op::PREFETCH) {
                // rows past the tile re-load the tile's last row (valid, unused)
#pragma unroll
                for (int u = 0; u < kPRE; ++u) pre[u] = op.load(min(r0 + tid + u * kWG, r1 - 1));
            }
            // the tile's row pointers, staged in LDS for phase 2
            int rpv[kRPT];
#pragma unroll
            for (int u = 0; u < kRPT; ++u) rpv[u] = rp[min(r0 + tid + u * kWG, r1 - 1)];
            if (cnt > 0) {  // uniform: a tile of empty rows has no nonzeros to stream
                typename Op::Raw raw[kEPT];
#pragma unroll
                for (int u = 0; u < kEPT; ++u) raw[u] = op.raw(P0 + min(tid + u * kWG, cnt - 1));
                int slot[kEPT];
#pragma unroll
                for (int u = 0; u < kEPT; ++u)
                    slot[u] = POS ? (int)__builtin_nontemporal_load(pos + P0 + min(tid + u * kWG, cnt - 1))
                                  : tid + u * kWG;
                S v[kEPT];
#pragma unroll
                for (int u = 0; u < kEPT; ++u) v[u] = op.prod(raw[u]);
#pragma unroll
                for (int u = 0; u < kEPT; ++u) {
                    const int k = tid + u * kWG;
                    if (k < cnt) prod[slot[u]] = v[u];
                }
            }
#pragma unroll
            for (int u = 0; u < kRPT; ++u) {
                const int rr = tid + u * kWG;
                if (rr < nrows) rpl[rr] = rpv[u] - P0;
            }
            if (tid == 0) rpl[nrows] = cnt;
            __syncthreads();
            int G = 1;
            while (G < 64 && 2 * G * nrows <= kWG) G <<= 1;
            const int lg = tid & (G - 1);
            const int ng = kWG / G;
            for (int rr = tid / G; rr < nrows; rr += ng) {
                const int b = rpl[rr], e = rpl[rr + 1];
                S s = szero<S>();
                for (int k = b + lg; k < e; k += G) s = s + prod[k];
                for (int off = G >> 1; off > 0; off >>= 1) s = s + xshfl(s, off);
                if (lg == 0) rsum[rr] = s;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < kRPT; ++u) {
                const int rr = tid + u * kWG;
                if (rr < nrows && ctx.active) {
                    if constexpr (Op::PREFETCH) {
                        if (u < kPRE) op.apply(r0 + rr, rsum[rr], pre[u < kPRE ? u : 0], ctx, q);
                        else op.apply(r0 + rr, rsum[rr], op.load(r0 + rr), ctx, q);
                    } else {
                        op.apply(r0 + rr, rsum[rr], op.load(r0 + rr), ctx, q);
                    }
                }
            }
        }
    } else if (kind == IT_ROW) {
        const int r = it.x;
        const PassCtx ctx = op.begin(it.w >> kKindBits);
        Pre pre{};
        if (Op::PREFETCH && tid == 0) pre = op.load(r);
        S s = row_sum(op, it.y, it.z, tid);
        s = block_sum(s, red);
        if (tid == 0 && ctx.active) op.apply(r, s, Op::PREFETCH ? pre : op.load(r), ctx, q);
    } else if (kind == IT_CHUNK) {
        // the partial of a stopped instance's chunk is written but never used (its split row
        // is not finished)
        S s = row_sum(op, it.x, it.y, tid);
        s = block_sum(s, red);
        if (tid == 0) split_part[it.w >> kKindBits] = s;
    } else if (kind == IT_BUNDLE) {
        // entries [k0, k0 + kn) of the R rows of a bundle, stored k-major from p = it.y:
        // entry kk of row l at p + kk R + l.  Lane l takes row l; wavefront w sums the entries
        // kk = w, w + 4, ... in increasing kk (kEPT loads in flight, out-of-range slots re-load
        // a valid entry and add zero), and the four wavefronts' sums are added in order.
        const int R = ((it.w >> kKindBits) & 63) + 1, kn = ((it.w >> 9) & 255) + 1;
        const int C = it.w >> 17;
        const int lane = tid & 63, wv = tid >> 6, l = min(lane, R - 1);
        S s = szero<S>();
        for (int k0 = wv; k0 < kn; k0 += 4 * kEPT) {
            typename Op::Raw raw[kEPT];
#pragma unroll
            for (int u = 0; u < kEPT; ++u) raw[u] = op.raw(it.y + min(k0 + 4 * u, kn - 1) * R + l);
            S v[kEPT];
#pragma unroll
            for (int u = 0; u < kEPT; ++u) v[u] = op.prod(raw[u]);
#pragma unroll
            for (int u = 0; u < kEPT; ++u) s = s + (k0 + 4 * u < kn ? v[u] : szero<S>());
        }
        S *bsum = reinterpret_cast<S *>(smem);  // [4][64]
        bsum[wv * 64 + lane] = s;
        __syncthreads();
        if (C == 1) {  // the whole rows: their epilogue here, lane l for row r0 + l
            const PassCtx ctx = op.begin(it.z);
            if (wv == 0 && lane < R && ctx.active) {
                const S tot = ((bsum[lane] + bsum[64 + lane]) + bsum[128 + lane]) + bsum[192 + lane];
                op.apply(it.x + lane, tot, op.load(it.x + lane), ctx, q);
            }
        } else if (wv == 0 && lane < R) {
            split_part[it.z + lane * C] =
                ((bsum[lane] + bsum[64 + lane]) + bsum[128 + lane]) + bsum[192 + lane];
        }
    }  // IT_EMPTY: padding item, only the (zero) check partials below
    if constexpr (Op::NQ > 0) {
#pragma unroll
        for (int j = 0; j < Op::NQ; ++j) {
            const double t = block_sum(q[j], redq);
            if (tid == 0) parts[(size_t)blockIdx.x * Op::NQ + j] = t;
        }
    }
}

// Column order of the nonzeros inside every tile (to_col), or back to row order.  In column
// order the gathers of one wavefront walk the gathered vector in increasing address order,
// so neighbouring lanes share cache lines; pos[p] keeps the row-order offset of the nonzero
// stored at p, which k_pass uses to stage each product in its row-order slot.  Ties (one
// column in several rows of the tile) keep row order.  One workgroup per item; other item
// kinds keep row order.
template <class M>
__global__ __launch_bounds__(kWG) void k_tile_order(const int4 *__restrict__ items,
                                                    int *__restrict__ ci, M *__restrict__ va,
                                                    unsigned short *__restrict__ pos,
                                                    int to_col) {
    __shared__ unsigned long long key[kMaxTileNnz];
    __shared__ M val[kMaxTileNnz];
    const int4 it = items[blockIdx.x];
    if ((it.w & kKindMask) != IT_TILE) return;
    const int P0 = it.y, cnt = (it.w >> kKindBits) & 4095;
    const int tid = threadIdx.x;
    if (to_col) {
        int N = 1;
        while (N < cnt) N <<= 1;
        for (int k = tid; k < N; k += kWG) {
            key[k] = k < cnt ? ((unsigned long long)(unsigned)ci[P0 + k] << 12) | (unsigned)k
                             : ~0ull;
            if (k < cnt) val[k] = va[P0 + k];
        }
        __syncthreads();
        for (int size = 2; size <= N; size <<= 1)  // bitonic sort of key[0, N)
            for (int stride = size >> 1; stride > 0; stride >>= 1) {
                for (int i = tid; i < N; i += kWG) {
                    const int j = i ^ stride;
                    if (j > i) {
                        const bool up = (i & size) == 0;
                        const unsigned long long a = key[i], b = key[j];
                        if ((a > b) == up) {
                            key[i] = b;
                            key[j] = a;
                        }
                    }
                }
                __syncthreads();
            }
        for (int q = tid; q < cnt; q += kWG) {
            const int k = (int)(key[q] & 4095ull);
            ci[P0 + q] = (int)(key[q] >> 12);
            va[P0 + q] = val[k];
            pos[P0 + q] = (unsigned short)k;
        }
    } else {
        for (int q = tid; q < cnt; q += kWG) {
            const int k = pos[P0 + q];
            key[k] = (unsigned long long)(unsigned)ci[P0 + q];
            val[k] = va[P0 + q];
        }
        __syncthreads();
        for (int k = tid; k < cnt; k += kWG) {
            ci[P0 + k] = (int)key[k];
            va[P0 + k] = val[k];
        }
    }
}

// Finish split rows: one wavefront per split row sums its slots in index order.
template <class Op>
__global__ __launch_bounds__(64) void k_split(const int4 *__restrict__ splits,
                                              const typename Op::Sum *__restrict__ part, Op op,
                                              double *__restrict__ parts, int slot_base) {
    using S = typename Op::Sum;
    constexpr int NQ = Op::NQ > 0 ? Op::NQ : 1;
    const int4 sp = splits[blockIdx.x];
    const PassCtx ctx = op.begin(sp.w);
    double q[NQ];
#pragma unroll
    for (int j = 0; j < NQ; ++j) q[j] = 0.0;
    if (ctx.active) {
        S s = szero<S>();
        for (int k = threadIdx.x; k < sp.z; k += 64) s = s + part[sp.y + k];
        s = wave_sum(s);
        if (threadIdx.x == 0) op.apply(sp.x, s, op.load(sp.x), ctx, q);
    }
    if constexpr (Op::NQ > 0) {
        if (threadIdx.x == 0) {
#pragma unroll
            for (int j = 0; j < Op::NQ; ++j)
                parts[(size_t)(slot_base + blockIdx.x) * Op::NQ + j] = q[j];
        }
    }
}

constexpr int kRedWG = 1024;

// Sum over a 1024-thread workgroup (16 wavefronts); valid in thread 0.
__device__ __forceinline__ double block_sum_1024(double v, double *red) {
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    double t = 0.0;
    if (threadIdx.x == 0)
        for (int w = 0; w < kRedWG / 64; ++w) t += red[w];
    return t;
}

// Fixed-order reduction of per-workgroup partials: out[j] = sum_k parts[k*nq + j].
__global__ __launch_bounds__(kRedWG) void k_reduce(const double *__restrict__ parts, int nslots,
                                                   int nq, double *__restrict__ out) {
    __shared__ double red[kRedWG / 64];
    for (int j = 0; j < nq; ++j) {
        double s = 0.0;
        for (int k = threadIdx.x; k < nslots; k += kRedWG) s += parts[(size_t)k * nq + j];
        s = block_sum_1024(s, red);
        if (threadIdx.x == 0) out[j] = s;
    }
}

// Segmented fixed-order reduction, one workgroup per instance b:
// out[b * out_stride + j] = sum over the slots of b (in slot order) of parts[slot*nq + j].
__global__ __launch_bounds__(kWG) void k_seg_reduce(const double *__restrict__ parts, int nq,
                                                    const int *__restrict__ ptr,
                                                    const int *__restrict__ slots,
                                                    double *__restrict__ out, int out_stride) {
    __shared__ double red[4];
    const int b = blockIdx.x;
    const int s0 = ptr[b], s1 = ptr[b + 1];
    for (int j = 0; j < nq; ++j) {
        double s = 0.0;
        for (int k = s0 + threadIdx.x; k < s1; k += kWG) s += parts[(size_t)slots[k] * nq + j];
        s = block_sum(s, red);
        if (threadIdx.x == 0) out[(size_t)b * out_stride + j] = s;
    }
}

// ------------------------------------------------------------------------- epilogues

// x-step over A^T (eqs. update-z/x): rows of A^T are the columns j of A.
//   x      = hx0 x0 + hx1 x_hat                 (x^{r,t}, rebuilt from the Halpern anchor)
//   v      = x + sigma * s_j (g - c)             (s_j = dc_j^2 when the scaling is folded)
//   x_bar  = Pi_C(v);   x_hat <- 2 x_bar - x     (gathered by the y-step)
//   relaxation rho != 2: x_rel <- rho x_bar + (1 - rho) x is the Halpern point, and the next
//   x is rebuilt from x_rel (x_rel = x_hat when rho = 2)
//   keep:  x_bar, z_int = (x_bar - v)/sigma (eq. update-z), dx = x - (relaxed point)
template <class M, class V, bool FOLD, bool KEEP, bool B> struct ColOp {
    using Sum = typename AccT<M, V>::type;
    using Raw = RawT<M>;
    static constexpr int NQ = 0;
    static constexpr bool PREFETCH = true;
    struct Pre {
        V xh, x0, cd, ld, ud, sc;
    };
    const int *__restrict__ ci;
    const M *__restrict__ va;
    const V *__restrict__ yg;
    V *__restrict__ xhat;
    V *__restrict__ xrel;  // nullptr when rho = 2
    const V *__restrict__ x0;
    const V *__restrict__ cd;
    const V *__restrict__ ld;
    const V *__restrict__ ud;
    const V *__restrict__ sc;
    V *__restrict__ xbar;
    V *__restrict__ zint;
    V *__restrict__ dx;
    IterScalars s;
    BatchArgs ba;
    __device__ __forceinline__ PassCtx begin(int inst) const {
        return B ? ctx_batch(ba, inst) : ctx_single(s, nullptr);
    }
    __device__ __forceinline__ Raw raw(int p) const { return load_raw(ci, va, p); }
    __device__ __forceinline__ Sum prod(const Raw &r) const { return (Sum)r.a * (Sum)yg[r.j]; }
    __device__ __forceinline__ Pre load(int j) const {
        return Pre{ep_load((xrel ? xrel : xhat) + j), ep_load(x0 + j), ep_load(cd + j),
                   ep_load(ld + j), ep_load(ud + j), FOLD ? ep_load(sc + j) : (V)1};
    }
    __device__ __forceinline__ void apply(int j, Sum g, const Pre &p, const PassCtx &c,
                                          double *) const {
        const V sigma = (V)c.sigma;
        const V x = (V)c.hx0 * p.x0 + (V)c.hx1 * p.xh;
        V gs = (V)g - p.cd;
        if (FOLD) gs = p.sc * gs;
        const V v = x + sigma * gs;
        const V xb = clampv(v, p.ld, p.ud);
        const V xr = (V)2 * xb - x;
        ep_store(xhat + j, xr);
        V xh = xr;
        if (xrel) {  // uniform
            xh = (V)c.rho * xb + ((V)1 - (V)c.rho) * x;
            xrel[j] = xh;
        }
        if (KEEP) {
            xbar[j] = xb;
            zint[j] = (xb - v) / sigma;
            dx[j] = x - xh;
        }
    }
};

// y-step over A (eq. update-y-2 with T1 = lambda I - A A^T):
//   y_bar = y + r_i (b - A x_hat)/(lambda sigma)  (r_i = dr_i^2 when folded);
//   y_bar = max(y_bar, 0) on inequality rows;   y <- hy0 y0 + hy1 (2 y_bar - y)
//   keep:  y_bar, dy = y - y_hat
template <class M, class V, bool FOLD, bool KEEP, bool B> struct RowOp {
    using Sum = typename AccT<M, V>::type;
    using Raw = RawT<M>;
    static constexpr int NQ = 0;
    static constexpr bool PREFETCH = true;
    struct Pre {
        V y, y0, bd, sr;
    };
    const int *__restrict__ ci;
    const M *__restrict__ va;
    const V *__restrict__ xg;
    V *__restrict__ y;
    const V *__restrict__ y0;
    const V *__restrict__ bd;
    const V *__restrict__ sr;
    V *__restrict__ ybar;
    V *__restrict__ dy;
    IterScalars s;
    BatchArgs ba;
    __device__ __forceinline__ PassCtx begin(int inst) const {
        return B ? ctx_batch(ba, inst) : ctx_single(s, nullptr);
    }
    __device__ __forceinline__ Raw raw(int p) const { return load_raw(ci, va, p); }
    __device__ __forceinline__ Sum prod(const Raw &r) const { return (Sum)r.a * (Sum)xg[r.j]; }
    __device__ __forceinline__ Pre load(int i) const {
        return Pre{y[i], y0[i], bd[i], FOLD ? sr[i] : (V)1};
    }
    __device__ __forceinline__ void apply(int i, Sum s_, const Pre &p, const PassCtx &c,
                                          double *) const {
        V r = p.bd - (V)s_;
        if (FOLD) r = p.sr * r;
        V yb = p.y + r / (V)c.lam_sigma;
        if (i >= c.m1_end) yb = vmax(yb, (V)0);
        // relaxed point rho y_bar + (1 - rho) y (2 y_bar - y for rho = 2)
        const V yr = c.rho == 2.0 ? (V)2 * yb - p.y : (V)c.rho * yb + ((V)1 - (V)c.rho) * p.y;
        y[i] = (V)c.hy0 * p.y0 + (V)c.hy1 * yr;
        if (KEEP) {
            ybar[i] = yb;
            dy[i] = p.y - yr;
        }
    }
};

// Residual of the T1 = 0 y-step (Section 3.2, item 1): r = b~ - A~ x_hat, the right-hand
// side that the dense inverse of A~A~^T is applied to.
struct T1ResidOp {
    using Sum = double;
    using Raw = RawT<double>;
    static constexpr int NQ = 0;
    static constexpr bool PREFETCH = true;
    struct Pre {
        double bd;
    };
    const int *__restrict__ ci;
    const double *__restrict__ va;
    const double *__restrict__ xg;
    const double *__restrict__ bd;
    double *__restrict__ r;
    IterScalars s;
    __device__ __forceinline__ PassCtx begin(int) const { return ctx_single(s, nullptr); }
    __device__ __forceinline__ Raw raw(int p) const { return load_raw(ci, va, p); }
    __device__ __forceinline__ Sum prod(const Raw &q) const { return q.a * xg[q.j]; }
    __device__ __forceinline__ Pre load(int i) const { return Pre{bd[i]}; }
    __device__ __forceinline__ void apply(int i, Sum s_, const Pre &p, const PassCtx &,
                                          double *) const {
        r[i] = p.bd - s_;
    }
};

// ------------------------------------------------------------------ MIXED, FP32 phase
//
// The FP32 phase keeps the iterate as FP32 displacements from the FP64 anchor w^{r,0} of
// the current outer loop of Algorithm 2 (the Halpern anchor, renewed at every restart), so
// FP32 resolution applies to the distance travelled since the last restart, not to |w|:
// the dual step (b - A x_hat) / (lambda sigma) stays representable when sigma is large.
// At every restart the FP64 anchor passes below store, in FP32,
//   q0 = sc (A^T y0 - c),  dl = l - x0,  du = u - x0   (columns)
//   r0 = sr (b - A x0),    ny0 = -y0                   (rows)
// and with d* = * - anchor the two half-steps (eqs. update-z/x and update-y-2) read
//   x-step: dx = hx1 dxh;  dv = dx + sigma (q0 + sc A^T dy);  dxb = clamp(dv, dl, du);
//           dxh <- 2 dxb - dx (the y-step gathers it)
//   y-step: dyb = dy + (r0 - sr A dxh) / (lambda sigma), max(dyb, ny0) on inequality rows;
//           dy <- hy1 (2 dyb - dy)
// since the Halpern weights sum to one (x - x0 = hx1 (x_hat - x0), y' - y0 = hy1 (y_hat -
// y0)).  The iterations that keep w_bar write x_bar = x0 + dxb, z = (dxb - dv) / sigma, dx,
// y_bar = y0 + dyb and dy in FP64, for the checks, which always run in FP64 (z_bar from the
// FP64 copy of q0).
template <bool KEEP, bool B> struct DColOp {
    using Sum = float;
    using Raw = RawT<float>;
    static constexpr int NQ = 0;
    static constexpr bool PREFETCH = true;
    struct Pre {
        float xh, q0, dl, du, sc;
    };
    const int *__restrict__ ci;
    const float *__restrict__ va;
    const float *__restrict__ dyg;
    float *__restrict__ dxh;
    float *__restrict__ dxrel;  // nullptr when rho = 2
    const float *__restrict__ q0;
    const float *__restrict__ dl;
    const float *__restrict__ du;
    const float *__restrict__ sc;
    const double *__restrict__ x0;
    const double *__restrict__ q0d;
    double *__restrict__ xbar;
    double *__restrict__ zint;
    double *__restrict__ dx;
    IterScalars s;
    BatchArgs ba;
    __device__ __forceinline__ PassCtx begin(int inst) const {
        return B ? ctx_batch(ba, inst) : ctx_single(s, nullptr);
    }
    __device__ __forceinline__ Raw raw(int p) const { return load_raw(ci, va, p); }
    __device__ __forceinline__ Sum prod(const Raw &r) const { return r.a * dyg[r.j]; }
    __device__ __forceinline__ Pre load(int j) const {
        return Pre{(dxrel ? dxrel : dxh)[j], q0[j], dl[j], du[j], sc[j]};
    }
    __device__ __forceinline__ void apply(int j, Sum g, const Pre &p, const PassCtx &c,
                                          double *) const {
        const float sigma = (float)c.sigma;
        const float d = (float)c.hx1 * p.xh;
        const float dv = d + sigma * (p.q0 + p.sc * g);
        const float db = clampv(dv, p.dl, p.du);
        const float dr = 2.f * db - d;
        dxh[j] = dr;
        float dh = dr;
        if (dxrel) {  // uniform
            dh = (float)c.rho * db + (1.f - (float)c.rho) * d;
            dxrel[j] = dh;
        }
        if (KEEP) {
            // z_bar = (x_bar - v) / sigma (eq. update-z): 0 where the projection left v
            // inside the box; at an active bound (dxb - dx) / sigma - (q0 + sc A^T dy) in FP64
            // with the FP64 q0 (in FP32, dxb - dv cancels to the rounding of sigma q0), with
            // the sign of the active bound kept
            double z = 0.0;
            if (db != dv) {
                z = ((double)db - (double)d) / c.sigma - (q0d[j] + (double)p.sc * (double)g);
                if (db == p.dl && db != p.du) z = z > 0.0 ? z : 0.0;
                else if (db == p.du && db != p.dl) z = z < 0.0 ? z : 0.0;
            }
            xbar[j] = x0[j] + (double)db;
            zint[j] = z;
            dx[j] = (double)(d - dh);
        }
    }
};

template <bool KEEP, bool B> struct DRowOp {
    using Sum = float;
    using Raw = RawT<float>;
    static constexpr int NQ = 0;
    static constexpr bool PREFETCH = true;
    struct Pre {
        float dy, r0, sr, ny0;
    };
    const int *__restrict__ ci;
    const float *__restrict__ va;
    const float *__restrict__ dxg;
    float *__restrict__ dy;
    const float *__restrict__ r0;
    const float *__restrict__ sr;
    const float *__restrict__ ny0;
    const double *__restrict__ y0;
    double *__restrict__ ybar;
    double *__restrict__ dyk;
    IterScalars s;
    BatchArgs ba;
    __device__ __forceinline__ PassCtx begin(int inst) const {
        return B ? ctx_batch(ba, inst) : ctx_single(s, nullptr);
    }
    __device__ __forceinline__ Raw raw(int p) const { return load_raw(ci, va, p); }
    __device__ __forceinline__ Sum prod(const Raw &r) const { return r.a * dxg[r.j]; }
    __device__ __forceinline__ Pre load(int i) const { return Pre{dy[i], r0[i], sr[i], ny0[i]}; }
    __device__ __forceinline__ void apply(int i, Sum s_, const Pre &p, const PassCtx &c,
                                          double *) const {
        const float r = p.r0 - p.sr * s_;
        float db = p.dy + r / (float)c.lam_sigma;
        if (i >= c.m1_end) db = vmax(db, p.ny0);
        const float dr = c.rho == 2.0 ? 2.f * db - p.dy
                                      : (float)c.rho * db + (1.f - (float)c.rho) * p.dy;
        dy[i] = (float)c.hy1 * dr;
        if (KEEP) {
            ybar[i] = y0[i] + (double)db;
            dyk[i] = (double)(p.dy - dr);
        }
    }
};

// The per-restart FP32 data of the displacement form, computed in FP64 from the anchor
// (A stored in FP32, FP32 x FP64 products exact in FP64).  Every row / column is written,
// stopped instances included (their anchor does not move, so their values do not change).
__device__ __forceinline__ PassCtx ctx_all() {
    PassCtx c{};
    c.active = 1;
    return c;
}

struct AnchorColOp {
    using Sum = double;
    using Raw = RawT<float>;
    using Pre = NoPre;
    static constexpr int NQ = 0;
    static constexpr bool PREFETCH = false;
    const int *__restrict__ ci;
    const float *__restrict__ va;
    const double *__restrict__ y0;
    const double *__restrict__ cd;
    const double *__restrict__ sc;
    const double *__restrict__ ld;
    const double *__restrict__ ud;
    const double *__restrict__ x0;
    float *__restrict__ q0;
    double *__restrict__ q0d;
    float *__restrict__ dl;
    float *__restrict__ du;
    __device__ __forceinline__ PassCtx begin(int) const { return ctx_all(); }
    __device__ __forceinline__ Raw raw(int p) const { return load_raw(ci, va, p); }
    __device__ __forceinline__ Sum prod(const Raw &r) const { return (double)r.a * y0[r.j]; }
    __device__ __forceinline__ Pre load(int) const { return Pre{}; }
    __device__ __forceinline__ void apply(int j, Sum g, const Pre &, const PassCtx &,
                                          double *) const {
        const double q = sc[j] * (g - cd[j]);
        q0d[j] = q;
        q0[j] = (float)q;
        dl[j] = (float)(ld[j] - x0[j]);
        du[j] = (float)(ud[j] - x0[j]);
    }
};

struct AnchorRowOp {
    using Sum = double;
    using Raw = RawT<float>;
    using Pre = NoPre;
    static constexpr int NQ = 0;
    static constexpr bool PREFETCH = false;
    const int *__restrict__ ci;
    const float *__restrict__ va;
    const double *__restrict__ x0;
    const double *__restrict__ bd;
    const double *__restrict__ sr;
    const double *__restrict__ y0;
    float *__restrict__ r0;
    float *__restrict__ ny0;
    __device__ __forceinline__ PassCtx begin(int) const { return ctx_all(); }
    __device__ __forceinline__ Raw raw(int p) const { return load_raw(ci, va, p); }
    __device__ __forceinline__ Sum prod(const Raw &r) const { return (double)r.a * x0[r.j]; }
    __device__ __forceinline__ Pre load(int) const { return Pre{}; }
    __device__ __forceinline__ void apply(int i, Sum s_, const Pre &, const PassCtx &,
                                          double *) const {
        r0[i] = (float)(sr[i] * (bd[i] - s_));
        ny0[i] = (float)(-y0[i]);
    }
};

// Check, row side (FP64): p = A x_bar and q = A dx from one pass over A.
//   q0 = ||Pi_D(b - A x)||^2 (original data)   q1 = same on the scaled data (sigma update)
//   q2 = <b, y_bar> / (beta_b beta_c)          q3 = ||dy||^2 (scaled)
//   q4 = <dy, A~ dx>                           q5 = ||y_bar - y0||^2 (scaled)
template <class M, class V, bool B> struct CheckRowOp {
    using Sum = D2;
    using Raw = RawT<M>;
    using Pre = NoPre;
    static constexpr int NQ = kNQ;
    static constexpr bool PREFETCH = false;
    const int *__restrict__ ci;
    const M *__restrict__ va;
    const V *__restrict__ xbar;
    const V *__restrict__ dxv;
    const V *__restrict__ ybar;
    const V *__restrict__ dyv;
    const V *__restrict__ y0;
    const double *__restrict__ bd;
    const double *__restrict__ ro;
    const double *__restrict__ rs;
    const double *__restrict__ ys;
    IterScalars s;
    BatchArgs ba;
    __device__ __forceinline__ PassCtx begin(int inst) const {
        return B ? ctx_batch(ba, inst) : ctx_single(s, nullptr);
    }
    __device__ __forceinline__ Raw raw(int p) const { return load_raw(ci, va, p); }
    __device__ __forceinline__ Sum prod(const Raw &r) const {
        const double a = (double)r.a;
        return D2{a * (double)xbar[r.j], a * (double)dxv[r.j]};
    }
    __device__ __forceinline__ Pre load(int) const { return Pre{}; }
    __device__ __forceinline__ void apply(int i, Sum s_, const Pre &, const PassCtx &c,
                                          double *q) const {
        const double e = bd[i] - s_.a;
        double eo = ro[i] * e, es = rs[i] * e;
        if (i >= c.m1_end) {
            eo = eo > 0.0 ? eo : 0.0;
            es = es > 0.0 ? es : 0.0;
        }
        q[0] += eo * eo;
        q[1] += es * es;
        const double yb = (double)ybar[i];
        q[2] += bd[i] * yb;
        const double dyi = (double)dyv[i];
        const double d = ys[i] * dyi;
        q[3] += d * d;
        q[4] += dyi * s_.b;
        const double e2 = ys[i] * (yb - (double)y0[i]);
        q[5] += e2 * e2;
    }
};

// Check, column side (FP64): g = A^T y_bar.
//   q0 = ||c - A^T y - z||^2 (original)   q1 = same on the scaled data
//   q2 = <c, x_bar> / (beta_b beta_c)     q3 = delta*_C(-z) (original, 0*inf := 0)
//   q4 = ||dx||^2 (scaled)                q5 = ||x_bar - x0||^2 (scaled)
template <class M, class V, bool FOLD, bool B> struct CheckColOp {
    using Sum = double;
    using Raw = RawT<M>;
    using Pre = NoPre;
    static constexpr int NQ = kNQ;
    static constexpr bool PREFETCH = false;
    const int *__restrict__ ci;
    const M *__restrict__ va;
    const V *__restrict__ ybar;
    const V *__restrict__ xbar;
    const V *__restrict__ zint;
    const V *__restrict__ dxv;
    const V *__restrict__ x0;
    const double *__restrict__ cd;
    const double *__restrict__ sc;
    const double *__restrict__ co;
    const double *__restrict__ cs;
    const double *__restrict__ xs;
    const double *__restrict__ lo;
    const double *__restrict__ uo;
    IterScalars s;
    BatchArgs ba;
    __device__ __forceinline__ PassCtx begin(int inst) const {
        return B ? ctx_batch(ba, inst) : ctx_single(s, nullptr);
    }
    __device__ __forceinline__ Raw raw(int p) const { return load_raw(ci, va, p); }
    __device__ __forceinline__ Sum prod(const Raw &r) const {
        return (double)r.a * (double)ybar[r.j];
    }
    __device__ __forceinline__ Pre load(int) const { return Pre{}; }
    __device__ __forceinline__ void apply(int j, Sum g, const Pre &, const PassCtx &,
                                          double *q) const {
        const double xb = (double)xbar[j];
        const double zi = (double)zint[j];
        double e = cd[j] - g;
        if (FOLD) e = sc[j] * e;
        e = e - zi;
        const double eo = co[j] * e, es = cs[j] * e;
        q[0] += eo * eo;
        q[1] += es * es;
        q[2] += cd[j] * xb;
        const double zo = co[j] * zi;
        double sup = 0.0;
        if (zo < 0.0) sup = -zo * uo[j];
        else if (zo > 0.0) sup = -zo * lo[j];
        q[3] += sup;
        const double d = xs[j] * (double)dxv[j];
        q[4] += d * d;
        const double e2 = xs[j] * (xb - (double)x0[j]);
        q[5] += e2 * e2;
    }
};

// Power method on A~ A~^T (Section 4.1), FP64.  With the scaling folded, the vectors that
// are gathered carry the diagonal factors: vg = D_r v, w = D_c A~^T v.
template <class M, bool FOLD, bool B> struct PowColOp {
    using Sum = double;
    using Raw = RawT<M>;
    using Pre = NoPre;
    static constexpr int NQ = 1;
    static constexpr bool PREFETCH = false;
    const int *__restrict__ ci;
    const M *__restrict__ va;
    const double *__restrict__ vg;
    const double *__restrict__ inv_norm;
    double *__restrict__ w;
    const double *__restrict__ sc;
    IterScalars s;
    BatchArgs ba;
    __device__ __forceinline__ PassCtx begin(int inst) const {
        return B ? ctx_batch(ba, inst) : ctx_single(s, inv_norm);
    }
    __device__ __forceinline__ Raw raw(int p) const { return load_raw(ci, va, p); }
    __device__ __forceinline__ Sum prod(const Raw &r) const { return (double)r.a * vg[r.j]; }
    __device__ __forceinline__ Pre load(int) const { return Pre{}; }
    __device__ __forceinline__ void apply(int j, Sum g, const Pre &, const PassCtx &c,
                                          double *q) const {
        const double gn = g * c.inv_norm;
        const double t = FOLD ? sc[j] * gn : gn;
        w[j] = t;
        q[0] += t * gn;  // ||A~^T v||^2
    }
};

template <class M, bool FOLD, bool B> struct PowRowOp {
    using Sum = double;
    using Raw = RawT<M>;
    using Pre = NoPre;
    static constexpr int NQ = 1;
    static constexpr bool PREFETCH = false;
    const int *__restrict__ ci;
    const M *__restrict__ va;
    const double *__restrict__ w;
    double *__restrict__ vg;
    const double *__restrict__ sr;
    IterScalars s;
    BatchArgs ba;
    __device__ __forceinline__ PassCtx begin(int inst) const {
        return B ? ctx_batch(ba, inst) : ctx_single(s, nullptr);
    }
    __device__ __forceinline__ Raw raw(int p) const { return load_raw(ci, va, p); }
    __device__ __forceinline__ Sum prod(const Raw &r) const { return (double)r.a * w[r.j]; }
    __device__ __forceinline__ Pre load(int) const { return Pre{}; }
    __device__ __forceinline__ void apply(int i, Sum s_, const Pre &, const PassCtx &,
                                          double *q) const {
        const double t = FOLD ? sr[i] * s_ : s_;
        vg[i] = t;
        q[0] += t * s_;  // ||A~ A~^T v||^2
    }
};

__global__ __launch_bounds__(kRedWG) void k_power_reduce(const double *__restrict__ pc, int nc,
                                                         const double *__restrict__ pr, int nr,
                                                         double *__restrict__ hist,
                                                         double *__restrict__ inv_norm) {
    __shared__ double red[kRedWG / 64];
    double s = 0.0;
    for (int k = threadIdx.x; k < nc; k += kRedWG) s += pc[k];
    s = block_sum_1024(s, red);
    double t = 0.0;
    for (int k = threadIdx.x; k < nr; k += kRedWG) t += pr[k];
    t = block_sum_1024(t, red);
    if (threadIdx.x == 0) {
        *hist = s;
        *inv_norm = t > 0.0 ? 1.0 / sqrt(t) : 0.0;
    }
}

// Batched power method: tmp[b] = ||A~_b^T v_b||^2, tmp[n + b] = ||A~_b A~_b^T v_b||^2.
__global__ void k_power_finish(const double *__restrict__ tmp, int n_inst,
                               double *__restrict__ hist_row, double *__restrict__ inv_norm) {
    const int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= n_inst) return;
    hist_row[b] = tmp[b];
    const double t = tmp[n_inst + b];
    inv_norm[b] = t > 0.0 ? 1.0 / sqrt(t) : 0.0;
}

// ------------------------------------------------------------------------- batched control

// One workgroup of 1024 threads takes the decisions of every instance after a chunk: the
// restart criteria of Section 3.1 on the merit R~ = ||w - w_hat||_M, SigmaUpdate (Algorithm 3
// with eq. sigma_T1!=0), and the termination test of Section 4.1 on the original data.  It is
// the device counterpart of the host loop of the single-LP solve, instance by instance.
__global__ __launch_bounds__(kRedWG) void k_decide(DecideArgs d) {
    __shared__ double red_a[kRedWG / 64], red_m[kRedWG / 64], red_s[kRedWG / 64];
    double n_active = 0.0, max_kkt = 0.0, n_switch = 0.0;
    const long long k0 = *d.kbase;          // iterations done before this chunk
    const long long k = k0 + d.chunk;       // iterations done after it
    for (int b = threadIdx.x; b < d.n_inst; b += kRedWG) {
        d.restart_flag[b] = 0;
        if (!d.active[b]) continue;
        const double *qf = d.res_first + (size_t)b * 2 * kNQ;   // row sums, then column sums
        const double *q = d.res_chk + (size_t)b * 2 * kNQ;
        const double *cst = d.cst + (size_t)b * 8;
        const double sigma = d.sigma[b], lam = d.lam[b];
        const double m_first = sqrt(fmax(sigma * lam * qf[3] + 2.0 * qf[4] + qf[kNQ + 4] / sigma, 0.0));
        const double merit = sqrt(fmax(sigma * lam * q[3] + 2.0 * q[4] + q[kNQ + 4] / sigma, 0.0));
        if (d.kstart[b] == k0) {  // this chunk began a new outer loop for b: R~_{r,0}
            d.merit0[b] = m_first;
            d.merit_prev[b] = m_first;
        }
        const double bbc = cst[0] * cst[1];
        const double rel_p = sqrt(q[0]) / (1.0 + cst[2]);
        const double rel_d = sqrt(q[kNQ + 0]) / (1.0 + cst[3]);
        const double pobj = bbc * q[kNQ + 2];
        const double dobj = bbc * q[2] - q[kNQ + 3];
        const double rel_gap = fabs(dobj - pobj) / (1.0 + fabs(dobj) + fabs(pobj));
        double kkt = rel_p > rel_d ? rel_p : rel_d;
        if (rel_gap > kkt) kkt = rel_gap;
        double *last = d.last + (size_t)b * 6;
        last[0] = rel_p; last[1] = rel_d; last[2] = rel_gap; last[3] = pobj; last[4] = dobj;
        last[5] = merit;
        const long long t = k - d.kstart[b];
        const long long nc = d.nchecks[b];
        double *tr = (nc < kTraceRows) ? d.trace + ((size_t)b * kTraceRows + nc) * kTraceCols : nullptr;
        if (tr) {
            tr[0] = (double)k; tr[1] = (double)t; tr[2] = (double)d.restarts[b]; tr[3] = sigma;
            tr[4] = merit; tr[5] = rel_p; tr[6] = rel_d; tr[7] = rel_gap; tr[8] = 0.0;
            tr[9] = sigma;
        }
        d.nchecks[b] = nc + 1;
        int st = 0;
        if (!(kkt == kkt)) st = HPRLP_NUMERICAL;
        else if (kkt <= d.tol) st = HPRLP_OPTIMAL;
        else if (k >= d.max_iter) st = HPRLP_ITER_LIMIT;
        if (st) {
            d.status[b] = st;
            d.active[b] = 0;
            d.iters_done[b] = k;
            continue;
        }
        bool restart = false;
        if (d.use_restart) {
            const double m0 = d.merit0[b];
            if (merit <= d.alpha1 * m0) restart = true;
            if (merit <= d.alpha2 * m0 && merit > d.merit_prev[b]) restart = true;
            if ((double)t >= d.alpha3 * (double)k) restart = true;
        }
        if (restart) {
            double sig_new = sigma;
            if (d.sigma_update) {
                const double Dx = sqrt(q[kNQ + 5]);
                const double Dy = sqrt(lam) * sqrt(q[5]);
                const double err_p = sqrt(q[1]) / (1.0 + cst[4]);
                const double err_d = sqrt(q[kNQ + 1]) / (1.0 + cst[5]);
                const bool ok = Dx > 1e-16 && Dx < 1e12 && Dy > 1e-16 && Dy < 1e12 &&
                                err_p > 0.0 && err_d / err_p > 1e-8 && err_d / err_p < 1e8;
                sig_new = ok ? Dx / Dy : 1.0;
            }
            d.sigma[b] = sig_new;
            d.kstart[b] = k;
            d.restarts[b] += 1;
            d.restart_flag[b] = 1;
            if (tr) { tr[8] = 1.0; tr[9] = sig_new; }
        } else {
            d.merit_prev[b] = merit;
        }
        n_active += 1.0;
        if (kkt > max_kkt) max_kkt = kkt;
        if (kkt > d.tol_switch) n_switch += 1.0;
    }
    // summary for the host: instances still iterating, their largest rel. KKT, how many of
    // them are still above the FP32 -> FP64 switch tolerance, iterations done
    const double v = wave_sum(n_active);
    const double w = wave_sum(n_switch);
    double mk = max_kkt;
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) {
        const double o = __shfl_xor(mk, off, 64);
        mk = o > mk ? o : mk;
    }
    if ((threadIdx.x & 63) == 0) {
        red_a[threadIdx.x >> 6] = v;
        red_m[threadIdx.x >> 6] = mk;
        red_s[threadIdx.x >> 6] = w;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double a = 0.0, m = 0.0, sw = 0.0;
        for (int i = 0; i < kRedWG / 64; ++i) {
            a += red_a[i];
            sw += red_s[i];
            m = red_m[i] > m ? red_m[i] : m;
        }
        d.summary[0] = a;
        d.summary[1] = m;
        d.summary[2] = sw;
        d.summary[3] = (double)k;
    }
}

// w^{r+1,0} = w_bar (anchors and current iterate) for the instances that restarted.
template <class V>
__global__ __launch_bounds__(kWG) void k_restart_batched(VecSet<V> v, const int *row_off,
                                                         const int *col_off,
                                                         const int *restart_flag) {
    const int b = blockIdx.x;
    if (!restart_flag[b]) return;
    for (int j = col_off[b] + threadIdx.x; j < col_off[b + 1]; j += kWG) {
        const V xb = v.xbar[j];
        v.x0[j] = xb;
        v.xhat[j] = xb;
        if (v.xrel) v.xrel[j] = xb;
    }
    for (int i = row_off[b] + threadIdx.x; i < row_off[b + 1]; i += kWG) {
        const V yb = v.ybar[i];
        v.y0[i] = yb;
        v.y[i] = yb;
    }
}

// Displacement form: w^{r+1,0} = w_bar (the FP64 anchor moves to the FP64 w_bar of the
// check) and the current iterate equals it (displacements zero).  One LP: grid-stride over
// all entries; batched: one workgroup per instance flagged by restart_flag.
__global__ void k_reanchor(DispSet v, long long n, long long m) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n; j += stride) {
        v.d.x0[j] = v.d.xbar[j];
        v.dxh[j] = 0.f;
        if (v.dxrel) v.dxrel[j] = 0.f;
    }
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m; i += stride) {
        v.d.y0[i] = v.d.ybar[i];
        v.dy[i] = 0.f;
    }
}

__global__ __launch_bounds__(kWG) void k_reanchor_batched(DispSet v, const int *row_off,
                                                          const int *col_off,
                                                          const int *restart_flag) {
    const int b = blockIdx.x;
    if (!restart_flag[b]) return;
    for (int j = col_off[b] + threadIdx.x; j < col_off[b + 1]; j += kWG) {
        v.d.x0[j] = v.d.xbar[j];
        v.dxh[j] = 0.f;
        if (v.dxrel) v.dxrel[j] = 0.f;
    }
    for (int i = row_off[b] + threadIdx.x; i < row_off[b + 1]; i += kWG) {
        v.d.y0[i] = v.d.ybar[i];
        v.dy[i] = 0.f;
    }
}

// Switch to FP64: x_hat, x_rel, y = anchor + displacement (the anchors and the kept w_bar
// are FP64 already).
__global__ void k_disp_promote(DispSet v, long long n, long long m) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long j = blockIdx.x * (long long)blockDim.x + threadIdx.x; j < n; j += stride) {
        const double x0 = v.d.x0[j];
        v.d.xhat[j] = x0 + (double)v.dxh[j];
        if (v.dxrel) v.d.xrel[j] = x0 + (double)v.dxrel[j];
    }
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < m; i += stride)
        v.d.y[i] = v.d.y0[i] + (double)v.dy[i];
}

__global__ void k_anchor_out(double *out, const double *a, const float *d, double h,
                             const double *mul, const int *perm, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[perm ? perm[i] : i] = mul[i] * (a[i] + h * (double)d[i]);
}

__global__ void k_advance(long long *kbase, int chunk) { *kbase += chunk; }

// ------------------------------------------------------------------------- launch helpers

template <class Op>
hipError_t run_pass(const DevMat &M, Op op, double *parts, hipStream_t st,
                    hipEvent_t ev_mid = nullptr) {
    using S = typename Op::Sum;
    // LDS: staged products (tile_nnz), row sums (tile_rows), row pointers (tile_rows + 1);
    // at least the four wavefronts' row sums of a bundle item
    const size_t lds = std::max((size_t)(M.tile_nnz + M.tile_rows) * sizeof(S) +
                                    (M.tile_rows + 1) * sizeof(int),
                                4 * 64 * sizeof(S));
    if (M.n_items > 0 && M.sorted)
        hipLaunchKernelGGL((k_pass<Op, true>), dim3(M.n_items), dim3(kWG), lds, st, M.items,
                           M.rp, op, reinterpret_cast<S *>(M.split_part), parts, M.tile_nnz,
                           M.tile_rows, M.pos);
    else if (M.n_items > 0)
        hipLaunchKernelGGL((k_pass<Op, false>), dim3(M.n_items), dim3(kWG), lds, st, M.items,
                           M.rp, op, reinterpret_cast<S *>(M.split_part), parts, M.tile_nnz,
                           M.tile_rows, nullptr);
    if (ev_mid) {
        hipError_t e = hipEventRecord(ev_mid, st);
        if (e != hipSuccess) return e;
    }
    if (M.n_split > 0)
        hipLaunchKernelGGL(k_split<Op>, dim3(M.n_split), dim3(64), 0, st, M.splits,
                           reinterpret_cast<const S *>(M.split_part), op, parts, M.n_items);
    return hipGetLastError();
}

template <class Op> void set_scalars(Op &op, const IterScalars &s, const BatchArgs *ba) {
    op.s = s;
    if (ba) op.ba = *ba;
}

template <class M, class V, bool FOLD, bool KEEP, bool B>
hipError_t col_pass(const DevMat &T, const VecSet<V> &v, const IterScalars &s, hipStream_t st,
                    hipEvent_t ev, const BatchArgs *ba) {
    ColOp<M, V, FOLD, KEEP, B> op;
    op.ci = T.ci;
    op.va = reinterpret_cast<const M *>(T.va);
    op.yg = v.y;
    op.xhat = v.xhat; op.xrel = v.xrel; op.x0 = v.x0; op.cd = v.cd; op.ld = v.ld; op.ud = v.ud;
    op.sc = v.sc; op.xbar = v.xbar; op.zint = v.zint; op.dx = v.dx;
    set_scalars(op, s, ba);
    return run_pass(T, op, nullptr, st, ev);
}

template <class M, class V, bool FOLD, bool KEEP, bool B>
hipError_t row_pass(const DevMat &A, const VecSet<V> &v, const IterScalars &s, hipStream_t st,
                    hipEvent_t ev, const BatchArgs *ba) {
    RowOp<M, V, FOLD, KEEP, B> op;
    op.ci = A.ci;
    op.va = reinterpret_cast<const M *>(A.va);
    op.xg = v.xhat;
    op.y = v.y; op.y0 = v.y0; op.bd = v.bd; op.sr = v.sr; op.ybar = v.ybar; op.dy = v.dy;
    set_scalars(op, s, ba);
    return run_pass(A, op, nullptr, st, ev);
}

template <bool KEEP, bool B>
hipError_t dcol_pass(const DevMat &T, const DispSet &v, const IterScalars &s, hipStream_t st,
                     hipEvent_t ev, const BatchArgs *ba) {
    DColOp<KEEP, B> op;
    op.ci = T.ci;
    op.va = reinterpret_cast<const float *>(T.va);
    op.dyg = v.dy;
    op.dxh = v.dxh; op.dxrel = v.dxrel; op.q0 = v.q0; op.dl = v.dl; op.du = v.du; op.sc = v.sc;
    op.x0 = v.d.x0; op.q0d = v.q0d; op.xbar = v.d.xbar; op.zint = v.d.zint; op.dx = v.d.dx;
    set_scalars(op, s, ba);
    return run_pass(T, op, nullptr, st, ev);
}

template <bool KEEP, bool B>
hipError_t drow_pass(const DevMat &A, const DispSet &v, const IterScalars &s, hipStream_t st,
                     hipEvent_t ev, const BatchArgs *ba) {
    DRowOp<KEEP, B> op;
    op.ci = A.ci;
    op.va = reinterpret_cast<const float *>(A.va);
    op.dxg = v.dxh;
    op.dy = v.dy; op.r0 = v.r0; op.sr = v.sr; op.ny0 = v.ny0;
    op.y0 = v.d.y0; op.ybar = v.d.ybar; op.dyk = v.d.dy;
    set_scalars(op, s, ba);
    return run_pass(A, op, nullptr, st, ev);
}

hipError_t reduce_parts(const DevMat &M, double *parts, int nq, double *out, hipStream_t st,
                        const Segments *seg, int out_stride) {
    if (seg) {
        if (seg->n_inst > 0)
            hipLaunchKernelGGL(k_seg_reduce, dim3(seg->n_inst), dim3(kWG), 0, st, parts, nq,
                               seg->ptr, seg->slots, out, out_stride);
    } else {
        hipLaunchKernelGGL(k_reduce, dim3(1), dim3(kRedWG), 0, st, parts,
                           M.n_items + M.n_split, nq, out);
    }
    return hipGetLastError();
}

template <class M, class V, bool B>
hipError_t check_row(const DevMat &A, const VecSet<V> &v, const CheckData &cd, const double *bd,
                     long long m1, double *parts, double *out, hipStream_t st,
                     const BatchArgs *ba, const Segments *seg, int out_stride) {
    CheckRowOp<M, V, B> op;
    op.ci = A.ci;
    op.va = reinterpret_cast<const M *>(A.va);
    op.xbar = v.xbar; op.dxv = v.dx; op.ybar = v.ybar; op.dyv = v.dy; op.y0 = v.y0;
    op.bd = bd; op.ro = cd.ro; op.rs = cd.rs; op.ys = cd.ys;
    IterScalars s{};
    s.m1 = m1;
    set_scalars(op, s, ba);
    hipError_t e = run_pass(A, op, parts, st);
    if (e != hipSuccess) return e;
    return reduce_parts(A, parts, kNQ, out, st, seg, out_stride);
}

template <class M, class V, bool FOLD, bool B>
hipError_t check_col(const DevMat &T, const VecSet<V> &v, const CheckData &cd, const double *cdv,
                     const double *sc, double *parts, double *out, hipStream_t st,
                     const BatchArgs *ba, const Segments *seg, int out_stride) {
    CheckColOp<M, V, FOLD, B> op;
    op.ci = T.ci;
    op.va = reinterpret_cast<const M *>(T.va);
    op.ybar = v.ybar; op.xbar = v.xbar; op.zint = v.zint; op.dxv = v.dx; op.x0 = v.x0;
    op.cd = cdv; op.sc = sc; op.co = cd.co; op.cs = cd.cs; op.xs = cd.xs;
    op.lo = cd.lo; op.uo = cd.uo;
    set_scalars(op, IterScalars{}, ba);
    hipError_t e = run_pass(T, op, parts, st);
    if (e != hipSuccess) return e;
    return reduce_parts(T, parts, kNQ, out, st, seg, out_stride);
}

template <class M, bool FOLD, bool B>
hipError_t power_iter(const DevMat &A, const DevMat &T, double *vg, double *w, const double *sc,
                      const double *sr, double *inv_norm, double *pc, double *pr, double *hist,
                      hipStream_t st, const BatchArgs *ba, const Segments *segA,
                      const Segments *segT, double *seg_tmp) {
    PowColOp<M, FOLD, B> oc;
    oc.ci = T.ci;
    oc.va = reinterpret_cast<const M *>(T.va);
    oc.vg = vg; oc.inv_norm = inv_norm; oc.w = w; oc.sc = sc;
    set_scalars(oc, IterScalars{}, ba);
    hipError_t e = run_pass(T, oc, pc, st);
    if (e != hipSuccess) return e;
    PowRowOp<M, FOLD, B> orw;
    orw.ci = A.ci;
    orw.va = reinterpret_cast<const M *>(A.va);
    orw.w = w; orw.vg = vg; orw.sr = sr;
    set_scalars(orw, IterScalars{}, ba);
    e = run_pass(A, orw, pr, st);
    if (e != hipSuccess) return e;
    if (!B) {
        hipLaunchKernelGGL(k_power_reduce, dim3(1), dim3(kRedWG), 0, st, pc,
                           T.n_items + T.n_split, pr, A.n_items + A.n_split, hist, inv_norm);
        return hipGetLastError();
    }
    const int n = segA->n_inst;
    if ((e = reduce_parts(T, pc, 1, seg_tmp, st, segT, 1)) != hipSuccess) return e;
    if ((e = reduce_parts(A, pr, 1, seg_tmp + n, st, segA, 1)) != hipSuccess) return e;
    hipLaunchKernelGGL(k_power_finish, dim3((n + 255) / 256), dim3(256), 0, st, seg_tmp, n,
                       hist, const_cast<double *>(ba->inv_norm));
    return hipGetLastError();
}

// ------------------------------------------------------------------------- vector kernels

template <class T> __global__ void k_fill(T *p, long long n, T v) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        p[i] = v;
}
template <class D, class S> __global__ void k_copy(D *dst, const S *src, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        dst[i] = (D)src[i];
}
template <class S>
__global__ void k_scale_out(double *out, const S *v, const double *mul, double smul,
                            const int *perm, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x)
        out[perm ? perm[i] : i] = (mul ? mul[i] : smul) * (double)v[i];
}
template <class S>
__global__ void k_xcur_out(double *out, const S *x0, const S *xh, double hx0, double hx1,
                           const double *mul, double smul, const int *perm, long long n) {
    for (long long i = blockIdx.x * (long long)blockDim.x + threadIdx.x; i < n;
         i += (long long)gridDim.x * blockDim.x) {
        const S x = (S)hx0 * x0[i] + (S)hx1 * xh[i];
        out[perm ? perm[i] : i] = (mul ? mul[i] : smul) * (double)x;
    }
}

inline dim3 grid_for(long long n) {
    long long g = (n + 255) / 256;
    if (g > 8192) g = 8192;
    if (g < 1) g = 1;
    return dim3((unsigned)g);
}

}  // namespace

// ------------------------------------------------------------------------- dispatch

#define HPRLP_PREC_DISPATCH(CALL)                                                               \
    do {                                                                                       \
        if (prec == 0) {                                                                       \
            auto &v = *static_cast<const VecSet<double> *>(vs);                                \
            return CALL(double, double, false);                                                \
        }                                                                                      \
        if (prec == 1) {                                                                       \
            auto &v = *static_cast<const VecSet<float> *>(vs);                                 \
            return CALL(float, float, true);                                                   \
        }                                                                                      \
        auto &v = *static_cast<const VecSet<double> *>(vs);                                    \
        return CALL(float, double, true);                                                      \
    } while (0)

hipError_t launch_col_pass(int prec, bool keep, const DevMat &T, const void *vs,
                           const IterScalars &s, hipStream_t st, hipEvent_t ev,
                           const BatchArgs *ba) {
    if (prec == 1) {
        const DispSet &v = *static_cast<const DispSet *>(vs);
        return ba ? (keep ? dcol_pass<true, true>(T, v, s, st, ev, ba)
                          : dcol_pass<false, true>(T, v, s, st, ev, ba))
                  : (keep ? dcol_pass<true, false>(T, v, s, st, ev, ba)
                          : dcol_pass<false, false>(T, v, s, st, ev, ba));
    }
#define COL_CALL(M, V, F)                                                                       \
    (ba ? (keep ? col_pass<M, V, F, true, true>(T, v, s, st, ev, ba)                           \
                : col_pass<M, V, F, false, true>(T, v, s, st, ev, ba))                         \
        : (keep ? col_pass<M, V, F, true, false>(T, v, s, st, ev, ba)                          \
                : col_pass<M, V, F, false, false>(T, v, s, st, ev, ba)))
    HPRLP_PREC_DISPATCH(COL_CALL);
#undef COL_CALL
}

hipError_t launch_t1_resid(const DevMat &A, const double *xhat, const double *bd, double *r,
                           hipStream_t st) {
    T1ResidOp op{A.ci, static_cast<const double *>(A.va), xhat, bd, r, IterScalars{}};
    return run_pass(A, op, nullptr, st);
}

hipError_t launch_row_pass(int prec, bool keep, const DevMat &A, const void *vs,
                           const IterScalars &s, hipStream_t st, hipEvent_t ev,
                           const BatchArgs *ba) {
    if (prec == 1) {
        const DispSet &v = *static_cast<const DispSet *>(vs);
        return ba ? (keep ? drow_pass<true, true>(A, v, s, st, ev, ba)
                          : drow_pass<false, true>(A, v, s, st, ev, ba))
                  : (keep ? drow_pass<true, false>(A, v, s, st, ev, ba)
                          : drow_pass<false, false>(A, v, s, st, ev, ba));
    }
#define ROW_CALL(M, V, F)                                                                       \
    (ba ? (keep ? row_pass<M, V, F, true, true>(A, v, s, st, ev, ba)                           \
                : row_pass<M, V, F, false, true>(A, v, s, st, ev, ba))                         \
        : (keep ? row_pass<M, V, F, true, false>(A, v, s, st, ev, ba)                          \
                : row_pass<M, V, F, false, false>(A, v, s, st, ev, ba)))
    HPRLP_PREC_DISPATCH(ROW_CALL);
#undef ROW_CALL
}

hipError_t launch_check_row(int prec, const DevMat &A, const void *vs, const CheckData &cd,
                            const double *bd64, long long m1, double *parts, double *out,
                            hipStream_t st, const BatchArgs *ba, const Segments *seg,
                            int out_stride) {
#define CR_CALL(M, V, F)                                                                        \
    (ba ? check_row<M, V, true>(A, v, cd, bd64, m1, parts, out, st, ba, seg, out_stride)       \
        : check_row<M, V, false>(A, v, cd, bd64, m1, parts, out, st, ba, seg, out_stride))
    HPRLP_PREC_DISPATCH(CR_CALL);
#undef CR_CALL
}

hipError_t launch_check_col(int prec, const DevMat &T, const void *vs, const CheckData &cd,
                            const double *cd64, const double *sc64, double *parts, double *out,
                            hipStream_t st, const BatchArgs *ba, const Segments *seg,
                            int out_stride) {
#define CC_CALL(M, V, F)                                                                        \
    (ba ? check_col<M, V, F, true>(T, v, cd, cd64, sc64, parts, out, st, ba, seg, out_stride)  \
        : check_col<M, V, F, false>(T, v, cd, cd64, sc64, parts, out, st, ba, seg, out_stride))
    HPRLP_PREC_DISPATCH(CC_CALL);
#undef CC_CALL
}

hipError_t launch_power_iter(bool mat_f32, bool fold, const DevMat &A, const DevMat &T,
                             double *vg, double *w, const double *sc, const double *sr,
                             double *inv_norm, double *pc, double *pr, double *hist, int k,
                             hipStream_t st, const BatchArgs *ba, const Segments *segA,
                             const Segments *segT, double *seg_tmp) {
    double *h = ba ? hist + (size_t)k * segA->n_inst : hist + k;
#define PW(M, F)                                                                                \
    (ba ? power_iter<M, F, true>(A, T, vg, w, sc, sr, inv_norm, pc, pr, h, st, ba, segA, segT,  \
                                 seg_tmp)                                                      \
        : power_iter<M, F, false>(A, T, vg, w, sc, sr, inv_norm, pc, pr, h, st, ba, segA,       \
                                  segT, seg_tmp))
    if (mat_f32) return fold ? PW(float, true) : PW(float, false);
    return fold ? PW(double, true) : PW(double, false);
#undef PW
}

hipError_t launch_decide(const DecideArgs &d, hipStream_t st) {
    hipLaunchKernelGGL(k_decide, dim3(1), dim3(kRedWG), 0, st, d);
    return hipGetLastError();
}

hipError_t launch_restart_batched(bool f32, const void *vs, const int *row_off,
                                  const int *col_off, const int *restart_flag, int n_inst,
                                  hipStream_t st) {
    if (n_inst <= 0) return hipSuccess;
    if (f32)
        hipLaunchKernelGGL(k_restart_batched<float>, dim3(n_inst), dim3(kWG), 0, st,
                           *static_cast<const VecSet<float> *>(vs), row_off, col_off,
                           restart_flag);
    else
        hipLaunchKernelGGL(k_restart_batched<double>, dim3(n_inst), dim3(kWG), 0, st,
                           *static_cast<const VecSet<double> *>(vs), row_off, col_off,
                           restart_flag);
    return hipGetLastError();
}

hipError_t launch_anchor(const DevMat &A, const DevMat &T, const DispSet &v, hipStream_t st) {
    AnchorColOp oc;
    oc.ci = T.ci;
    oc.va = reinterpret_cast<const float *>(T.va);
    oc.y0 = v.d.y0; oc.cd = v.d.cd; oc.sc = v.d.sc; oc.ld = v.d.ld; oc.ud = v.d.ud;
    oc.x0 = v.d.x0; oc.q0 = v.q0; oc.q0d = v.q0d; oc.dl = v.dl; oc.du = v.du;
    hipError_t e = run_pass(T, oc, nullptr, st);
    if (e != hipSuccess) return e;
    AnchorRowOp orw;
    orw.ci = A.ci;
    orw.va = reinterpret_cast<const float *>(A.va);
    orw.x0 = v.d.x0; orw.bd = v.d.bd; orw.sr = v.d.sr; orw.y0 = v.d.y0;
    orw.r0 = v.r0; orw.ny0 = v.ny0;
    return run_pass(A, orw, nullptr, st);
}

hipError_t launch_reanchor(const DispSet &v, long long n, long long m, hipStream_t st) {
    hipLaunchKernelGGL(k_reanchor, grid_for(n > m ? n : m), dim3(256), 0, st, v, n, m);
    return hipGetLastError();
}

hipError_t launch_reanchor_batched(const DispSet &v, const int *row_off, const int *col_off,
                                   const int *restart_flag, int n_inst, hipStream_t st) {
    if (n_inst > 0)
        hipLaunchKernelGGL(k_reanchor_batched, dim3(n_inst), dim3(kWG), 0, st, v, row_off,
                           col_off, restart_flag);
    return hipGetLastError();
}

hipError_t launch_disp_promote(const DispSet &v, long long n, long long m, hipStream_t st) {
    hipLaunchKernelGGL(k_disp_promote, grid_for(n > m ? n : m), dim3(256), 0, st, v, n, m);
    return hipGetLastError();
}

hipError_t launch_anchor_out(double *out, const double *a, const float *d, double h,
                             const double *mul, const int *perm, long long n, hipStream_t st) {
    hipLaunchKernelGGL(k_anchor_out, grid_for(n), dim3(256), 0, st, out, a, d, h, mul, perm, n);
    return hipGetLastError();
}

// Bundle storage: destination offset e = k R + l (entry k of row l) takes source l L + k.
template <class M>
__global__ void k_bundle_order(int *__restrict__ ci, M *__restrict__ va,
                               const int *__restrict__ tci, const M *__restrict__ tva,
                               long long P0, int R, int L) {
    const long long e = blockIdx.x * (long long)blockDim.x + threadIdx.x;
    if (e >= (long long)R * L) return;
    const long long src = (e % R) * (long long)L + e / R;
    ci[P0 + e] = tci[src];
    va[P0 + e] = tva[src];
}

hipError_t launch_bundle_order(int *ci, void *va, bool mat_f32, const int *tci, const void *tva,
                               long long P0, int R, int L, hipStream_t st) {
    const long long n = (long long)R * L;
    const dim3 grid((unsigned)((n + 255) / 256));
    if (mat_f32)
        hipLaunchKernelGGL(k_bundle_order<float>, grid, dim3(256), 0, st, ci,
                           static_cast<float *>(va), tci, static_cast<const float *>(tva), P0, R,
                           L);
    else
        hipLaunchKernelGGL(k_bundle_order<double>, grid, dim3(256), 0, st, ci,
                           static_cast<double *>(va), tci, static_cast<const double *>(tva), P0,
                           R, L);
    return hipGetLastError();
}

hipError_t launch_tile_order(const DevMat &M, bool mat_f32, bool to_col, hipStream_t st) {
    if (!M.pos || M.n_items == 0) return hipSuccess;
    if (mat_f32)
        hipLaunchKernelGGL(k_tile_order<float>, dim3(M.n_items), dim3(kWG), 0, st, M.items, M.ci,
                           static_cast<float *>(M.va), M.pos, to_col ? 1 : 0);
    else
        hipLaunchKernelGGL(k_tile_order<double>, dim3(M.n_items), dim3(kWG), 0, st, M.items,
                           M.ci, static_cast<double *>(M.va), M.pos, to_col ? 1 : 0);
    return hipGetLastError();
}

hipError_t launch_advance(long long *kbase, int chunk, hipStream_t st) {
    hipLaunchKernelGGL(k_advance, dim3(1), dim3(1), 0, st, kbase, chunk);
    return hipGetLastError();
}

hipError_t launch_fill(double *p, long long n, double v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<double>, grid_for(n), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t launch_fill_f(float *p, long long n, float v, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_fill<float>, grid_for(n), dim3(256), 0, st, p, n, v);
    return hipGetLastError();
}
hipError_t launch_copy_d(double *dst, const double *src, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_copy<double, double>), grid_for(n), dim3(256), 0, st, dst, src, n);
    return hipGetLastError();
}
hipError_t launch_copy_f(float *dst, const float *src, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_copy<float, float>), grid_for(n), dim3(256), 0, st, dst, src, n);
    return hipGetLastError();
}
hipError_t launch_f2d(double *dst, const float *src, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL((k_copy<double, float>), grid_for(n), dim3(256), 0, st, dst, src, n);
    return hipGetLastError();
}
hipError_t launch_scale_out(double *out, const void *v, bool v_f32, const double *mul,
                            double smul, const int *perm, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (v_f32)
        hipLaunchKernelGGL(k_scale_out<float>, grid_for(n), dim3(256), 0, st, out,
                           static_cast<const float *>(v), mul, smul, perm, n);
    else
        hipLaunchKernelGGL(k_scale_out<double>, grid_for(n), dim3(256), 0, st, out,
                           static_cast<const double *>(v), mul, smul, perm, n);
    return hipGetLastError();
}
hipError_t launch_xcur_out(double *out, const void *x0, const void *xhat, bool v_f32,
                           double hx0, double hx1, const double *mul, double smul,
                           const int *perm, long long n, hipStream_t st) {
    if (n <= 0) return hipSuccess;
    if (v_f32)
        hipLaunchKernelGGL(k_xcur_out<float>, grid_for(n), dim3(256), 0, st, out,
                           static_cast<const float *>(x0), static_cast<const float *>(xhat),
                           hx0, hx1, mul, smul, perm, n);
    else
        hipLaunchKernelGGL(k_xcur_out<double>, grid_for(n), dim3(256), 0, st, out,
                           static_cast<const double *>(x0), static_cast<const double *>(xhat),
                           hx0, hx1, mul, smul, perm, n);
    return hipGetLastError();
}

}  // namespace hprlp
