// The T1 = 0 variant of Section 3.2 (item 1) for LPs without inequality rows: the y-step
// is the exact minimiser of the augmented Lagrangian,
//     A~A~^T y_bar = (b~ - A~(x_bar + sigma (z_bar - c~))) / sigma        (eq. AATy=R),
// which, with the x-step, reads y_bar = y + G (b~ - A~ x_hat) / sigma, where G = (A~A~^T)^{-1}
// and x_hat = 2 x_bar - x.
//
// At create, G is formed once in the workspace, in place, in an mp x mp array (mp = m rounded
// up to 64; the padding is an identity block, so every tile is whole and the inverse's
// padding stays the identity):
//   * the dense Gram matrix A~A~^T, one wavefront per (row, 4096-column chunk), summed in
//     LDS in a fixed order;
//   * a blocked symmetric sweep (Gauss-Jordan elimination on the lower triangle, which needs
//     no pivoting on a positive definite matrix): for each panel P of 64 pivots, one
//     workgroup sweeps the diagonal block A_PP in LDS (its pivots are the LDL^T pivots of
//     A~A~^T, kept for the rank check), then V = A_{:,P} A_PP^{-1} (FP64 MFMA), then the
//     rank-64 update A_IJ -= V_I A_{J,P}^T of every lower tile (FP64 MFMA), which also writes
//     the panel's new row and column;
//   * the swept matrix is -G: one pass negates it and fills the upper triangle.
// Every iteration then costs one residual pass over A~ (the pass kernel with A's schedule,
// row bundles included) and one dense matrix-vector product with G (m^2 FP64 reads,
// HBM-bound), with the y epilogue of Algorithm 2 fused into it.  The
// checks need ||A~^T v||^2 (M of eq. def:M with T1 = 0, and eq. sigma_T1=0), from one pass
// over A~^T.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "hprlp_internal.h"

namespace hprlp {
namespace {

constexpr int kT = 256;        // threads per block of the row-wise and tile kernels
constexpr int kB = 64;         // panel width and tile edge of the dense inverse
constexpr int kLd = kB + 2;    // LDS row stride of a staged tile: MFMA operand reads hit
                               // 32 distinct 8-byte banks per half-wavefront
constexpr int kChunk = 4096;   // Gram columns one wavefront holds in LDS (32 KB)

typedef double d4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// broadcast of lane t's value (t uniform)
__device__ __forceinline__ int lane_int(int v, int t) { return __builtin_amdgcn_readlane(v, t); }
__device__ __forceinline__ double lane_dbl(double v, int t) {
    const long long w = __double_as_longlong(v);
    const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)w, t);
    const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(w >> 32), t);
    return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

// Columns [c0, c0 + kChunk) of row i of A~A~^T (blockIdx = (i, chunk)).  Row i's nonzeros
// are read 64 at a time, one per lane: column j, a_ij, the extent of A~^T row j and its
// first two entries.  Then, in storage order, each adds a_ij * (A~^T row j) into the LDS
// entries of its chunk: lanes 0 and 1 take the prefetched entries, longer columns loop over
// the rest.  The entries of one column are distinct rows and a wavefront issues its LDS
// accesses in program order, so every entry sums its terms in storage order.  Rows i >= m
// of the padding are identity rows.
__global__ __launch_bounds__(64) void k_gram(const int *__restrict__ rp,
                                             const int *__restrict__ ci,
                                             const double *__restrict__ va,
                                             const int *__restrict__ rpt,
                                             const int *__restrict__ cit,
                                             const double *__restrict__ vat, int m, int mp,
                                             double *__restrict__ F) {
    __shared__ double acc[kChunk];
    const int i = blockIdx.x, lane = threadIdx.x;
    const int c0 = blockIdx.y * kChunk;
    const int cn = min(kChunk, mp - c0);
    double *Fi = F + (int64_t)i * mp + c0;
    if (i >= m) {
        for (int k = lane; k < cn; k += 64) Fi[k] = c0 + k == i ? 1.0 : 0.0;
        return;
    }
    for (int k = lane; k < cn; k += 64) acc[k] = 0.0;
    __syncthreads();
    const int pe = rp[i + 1];
    for (int p0 = rp[i]; p0 < pe; p0 += 64) {
        const int p = p0 + lane;
        int s = 0, e = 0, k0 = -1, k1 = -1;
        double a = 0.0, v0 = 0.0, v1 = 0.0;
        if (p < pe) {
            const int j = ci[p];
            a = va[p];
            s = rpt[j];
            e = rpt[j + 1];
            if (e > s) { k0 = cit[s]; v0 = vat[s]; }
            if (e > s + 1) { k1 = cit[s + 1]; v1 = vat[s + 1]; }
        }
        const int cnt = min(64, pe - p0);
        for (int t = 0; t < cnt; ++t) {
            const double at = lane_dbl(a, t);
            const int ka = lane_int(k0, t), kb = lane_int(k1, t);
            const double wa = lane_dbl(v0, t), wb = lane_dbl(v1, t);
            const int kk = (lane == 0 ? ka : kb) - c0;
            if (lane < 2 && kk >= 0 && kk < cn) acc[kk] += at * (lane == 0 ? wa : wb);
            const int st = lane_int(s, t), et = lane_int(e, t);
            for (int q = st + 2 + lane; q < et; q += 64) {
                const int k = cit[q] - c0;
                if (k >= 0 && k < cn) acc[k] += at * vat[q];
            }
        }
    }
    __syncthreads();
    for (int k = lane; k < cn; k += 64) Fi[k] = acc[k];
}

__global__ void k_diag(const double *__restrict__ F, int m, int mp, double *__restrict__ d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) d[i] = F[(int64_t)i * mp + i];
}

// Sweeps the 64 pivots of the diagonal block at p0 (symmetrised from the lower triangle)
// in LDS, in order: with pivot d = S_kk, S_ij -= S_ik S_kj / d off row and column k, then
// row and column k are divided by d and S_kk = -1/d (by the reciprocal of d; two LDS
// copies alternate, so each pivot needs one barrier).  The pivots are the Schur complements
// of the whole matrix, i.e. its LDL^T pivots (to diagd); afterwards S = -A_PP^{-1}, and Sb
// receives A_PP^{-1}.
__global__ __launch_bounds__(kT) void k_sweep_diag(const double *__restrict__ F, int mp,
                                                   int p0, double *__restrict__ Sb,
                                                   double *__restrict__ diagd) {
    __shared__ double S[2][kB][kLd];
    const int t = threadIdx.x;
    const int b = t % kB, a0 = t / kB;  // this thread's entries: (a0 + 4s, b), s < 16
    constexpr int kPer = kB * kB / kT;
    for (int s = 0; s < kPer; ++s) {
        const int a = a0 + 4 * s;
        const int r = a > b ? a : b, c = a > b ? b : a;
        S[0][a][b] = F[(int64_t)(p0 + r) * mp + p0 + c];
    }
    __syncthreads();
    for (int k = 0; k < kB; ++k) {
        const double (*X)[kLd] = S[k & 1];
        double (*Y)[kLd] = S[(k & 1) ^ 1];
        const double d = X[k][k], rd = 1.0 / d;
        const double skb = X[k][b] * rd;
        for (int s = 0; s < kPer; ++s) {
            const int a = a0 + 4 * s;
            double v;
            if (a == k) v = b == k ? -rd : skb;
            else if (b == k) v = X[a][k] * rd;
            else v = X[a][b] - X[a][k] * skb;
            Y[a][b] = v;
        }
        if (t == 0) diagd[p0 + k] = d;
        __syncthreads();
    }
    for (int s = 0; s < kPer; ++s) {  // kB is even: the result is in S[0]
        const int a = a0 + 4 * s;
        Sb[a * kB + b] = -S[0][a][b];
    }
}

// Acc(32 x 32 corner (r0, c0) of a 64 x 64 tile) += X Y^T over k < 64, X and Y staged in LDS
// as [row][k]: 2 x 2 blocks of v_mfma_f64_16x16x4f64 per wavefront.  Lane l feeds
// X[r0 + 16 bi + l % 16][k0 + l / 16] and Y[c0 + 16 bj + l % 16][k0 + l / 16]; it holds the
// block's entries (l / 16 + 4 q, l % 16), q < 4.  neg: X enters negated.
__device__ __forceinline__ void tile_mma(const double (*X)[kLd], const double (*Y)[kLd],
                                         int r0, int c0, bool neg, d4 acc[2][2]) {
    const int lane = threadIdx.x & 63;
    const int lr = lane & 15, lk = lane >> 4;
    for (int k0 = 0; k0 < kB; k0 += 4) {
        double xa[2], yb[2];
        for (int bi = 0; bi < 2; ++bi) {
            const double x = X[r0 + 16 * bi + lr][k0 + lk];
            xa[bi] = neg ? -x : x;
        }
        for (int bj = 0; bj < 2; ++bj) yb[bj] = Y[c0 + 16 * bj + lr][k0 + lk];
        for (int bi = 0; bi < 2; ++bi)
            for (int bj = 0; bj < 2; ++bj)
                acc[bi][bj] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[bi], yb[bj], acc[bi][bj],
                                                                    0, 0, 0);
    }
}

// Block row I != P (blockIdx.x = I): U_I = A_{I,P} before the sweep of P (for I < P the
// transpose of the stored A_{P,I}) and V_I = U_I A_PP^{-1}, both stored compactly as
// [mp][64] (row I*64 + a).
__global__ __launch_bounds__(kT) void k_sweep_panel(const double *__restrict__ F, int mp,
                                                    int p0, const double *__restrict__ Sb,
                                                    double *__restrict__ U,
                                                    double *__restrict__ V) {
    const int I0 = blockIdx.x * kB;
    if (I0 == p0) return;
    __shared__ double u[kB][kLd], st[kB][kLd];
    const int t = threadIdx.x;
    for (int e = t; e < kB * kB; e += kT) {
        const int hi = e / kB, lo = e % kB;
        st[lo][hi] = Sb[e];  // st[c][k] = (A_PP^{-1})_{kc}
        if (I0 > p0) u[hi][lo] = F[(int64_t)(I0 + hi) * mp + p0 + lo];
        else u[lo][hi] = F[(int64_t)(p0 + hi) * mp + I0 + lo];
    }
    __syncthreads();
    for (int e = t; e < kB * kB; e += kT) U[(int64_t)(I0 + e / kB) * kB + e % kB] = u[e / kB][e % kB];
    const int w = t >> 6, lane = t & 63;
    const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
    d4 acc[2][2];
    for (int bi = 0; bi < 2; ++bi)
        for (int bj = 0; bj < 2; ++bj) acc[bi][bj] = d4{0.0, 0.0, 0.0, 0.0};
    tile_mma(u, st, r0, c0, false, acc);
    for (int bi = 0; bi < 2; ++bi)
        for (int bj = 0; bj < 2; ++bj)
            for (int q = 0; q < 4; ++q) {
                const int a = r0 + 16 * bi + (lane >> 4) + 4 * q, c = c0 + 16 * bj + (lane & 15);
                V[(int64_t)(I0 + a) * kB + c] = acc[bi][bj][q];
            }
}

// Lower tile number x -> (I, J), J <= I, row by row.
__device__ __forceinline__ void lower_tile(int x, int &I, int &J) {
    int i = (int)((sqrt(8.0 * (double)x + 1.0) - 1.0) * 0.5);
    while (i * (i + 1) / 2 > x) --i;
    while ((i + 1) * (i + 2) / 2 <= x) ++i;
    I = i;
    J = x - i * (i + 1) / 2;
}

// The sweep of panel P on lower tile (I, J) (blockIdx.x enumerates the lower tiles):
// A_IJ -= V_I U_J^T off the panel; the panel's tiles take their swept values
// (A_IP = V_I, A_PJ = V_J^T, A_PP = -A_PP^{-1}).
__global__ __launch_bounds__(kT) void k_sweep_update(double *__restrict__ F, int mp, int p0,
                                                     const double *__restrict__ Sb,
                                                     const double *__restrict__ U,
                                                     const double *__restrict__ V) {
    int I, J;
    lower_tile(blockIdx.x, I, J);
    const int I0 = I * kB, J0 = J * kB, t = threadIdx.x;
    if (I0 == p0 || J0 == p0) {
        for (int e = t; e < kB * kB; e += kT) {
            const int a = e / kB, b = e % kB;
            double v;
            if (I0 == p0 && J0 == p0) v = -Sb[e];
            else if (I0 == p0) v = V[(int64_t)(J0 + b) * kB + a];
            else v = V[(int64_t)(I0 + a) * kB + b];
            F[(int64_t)(I0 + a) * mp + J0 + b] = v;
        }
        return;
    }
    __shared__ double vi[kB][kLd], uj[kB][kLd];
    for (int e = t; e < kB * kB; e += kT) {
        const int a = e / kB, b = e % kB;
        vi[a][b] = V[(int64_t)(I0 + a) * kB + b];
        uj[a][b] = U[(int64_t)(J0 + a) * kB + b];
    }
    const int w = t >> 6, lane = t & 63;
    const int r0 = 32 * (w >> 1), c0 = 32 * (w & 1);
    d4 acc[2][2];
    double *Ft = F + (int64_t)I0 * mp + J0;
    for (int bi = 0; bi < 2; ++bi)
        for (int bj = 0; bj < 2; ++bj)
            for (int q = 0; q < 4; ++q) {
                const int a = r0 + 16 * bi + (lane >> 4) + 4 * q, c = c0 + 16 * bj + (lane & 15);
                acc[bi][bj][q] = Ft[(int64_t)a * mp + c];
            }
    __syncthreads();
    tile_mma(vi, uj, r0, c0, true, acc);
    for (int bi = 0; bi < 2; ++bi)
        for (int bj = 0; bj < 2; ++bj)
            for (int q = 0; q < 4; ++q) {
                const int a = r0 + 16 * bi + (lane >> 4) + 4 * q, c = c0 + 16 * bj + (lane & 15);
                Ft[(int64_t)a * mp + c] = acc[bi][bj][q];
            }
}

// G = -(swept matrix), symmetric from its lower triangle: lower tile (I, J) negated in place
// and, transposed, into the upper tile (J, I) (which nothing else reads).
__global__ __launch_bounds__(kT) void k_sweep_finish(double *__restrict__ F, int mp) {
    int I, J;
    lower_tile(blockIdx.x, I, J);
    const int I0 = I * kB, J0 = J * kB, t = threadIdx.x;
    __shared__ double tl[kB][kB + 1];
    for (int e = t; e < kB * kB; e += kT)
        tl[e / kB][e % kB] = F[(int64_t)(I0 + e / kB) * mp + J0 + e % kB];
    __syncthreads();
    for (int e = t; e < kB * kB; e += kT) {
        const int a = e / kB, b = e % kB;
        const double v = I != J || a >= b ? tl[a][b] : tl[b][a];
        F[(int64_t)(I0 + a) * mp + J0 + b] = -v;
        if (I != J) F[(int64_t)(J0 + a) * mp + I0 + b] = -tl[b][a];
    }
}

// y-step with T1 = 0 and the rest of Algorithm 2's y update, one wavefront per row:
// y_bar = y + (G r)_i / sigma; relaxed point rho y_bar + (1 - rho) y; Halpern average.
__global__ __launch_bounds__(kT) void k_t1_solve(const double *__restrict__ G,
                                                 const double *__restrict__ r, int m,
                                                 int ld, double *__restrict__ y,
                                                 const double *__restrict__ y0,
                                                 double *__restrict__ ybar,
                                                 double *__restrict__ dy, IterScalars s,
                                                 int keep) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    if (i >= m) return;
    const double *Gi = G + (int64_t)i * ld;
    // four partial sums keep four loads of the row in flight per lane (fixed order)
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
    int k = lane;
    for (; k + 192 < m; k += 256) {
        d0 += Gi[k] * r[k];
        d1 += Gi[k + 64] * r[k + 64];
        d2 += Gi[k + 128] * r[k + 128];
        d3 += Gi[k + 192] * r[k + 192];
    }
    for (; k < m; k += 64) d0 += Gi[k] * r[k];
    double d = wave_sum((d0 + d1) + (d2 + d3));
    if (lane != 0) return;
    const double yi = y[i];
    double yb = yi + d / s.sigma;
    if (i >= s.m1) yb = yb > 0.0 ? yb : 0.0;  // no inequality rows in this variant
    const double yr = s.rho == 2.0 ? 2.0 * yb - yi : s.rho * yb + (1.0 - s.rho) * yi;
    y[i] = s.hy0 * y0[i] + s.hy1 * yr;
    if (keep) {
        ybar[i] = yb;
        dy[i] = yi - yr;
    }
}

// G r from the lower triangle of G only (G beyond the infinity cache): lower tile (I, K)
// (blockIdx.x enumerates the lower tiles) gives the row partials G_IK r_K -> P[I0 + a][K]
// and, for K < I, the column partials (G_IK)^T r_I = G_KI r_I -> P[K0 + b][I].  Wavefront
// w takes the tile's rows a = w + 4j (j < 16, in order), lane b its column b; every
// partial has a fixed order (the row partial a butterfly over the lanes, the column
// partial the rows of each wavefront, then the four wavefronts in order).
__global__ __launch_bounds__(kT) void k_t1_gr_tiles(const double *__restrict__ G,
                                                    const double *__restrict__ r, int m,
                                                    int mp, int nbk, double *__restrict__ P) {
    int I, K;
    lower_tile(blockIdx.x, I, K);
    const int I0 = I * kB, K0 = K * kB, t = threadIdx.x, w = t >> 6, b = t & 63;
    __shared__ double colp[4][kB];
    const double rk = K0 + b < m ? r[K0 + b] : 0.0;
    double cacc = 0.0;
    for (int j = 0; j < kB / 4; ++j) {
        const int a = w + 4 * j;
        const double g = G[(int64_t)(I0 + a) * mp + K0 + b];
        const double ra = I0 + a < m ? r[I0 + a] : 0.0;
        const double s = wave_sum(g * rk);
        if (b == 0) P[(int64_t)(I0 + a) * nbk + K] = s;
        cacc += g * ra;
    }
    if (K < I) {
        colp[w][b] = cacc;
        __syncthreads();
        if (w == 0)
            P[(int64_t)(K0 + b) * nbk + I] = ((colp[0][b] + colp[1][b]) + colp[2][b]) + colp[3][b];
    }
}

// The y-step after k_t1_gr_tiles: (G r)_i = the sum of row i's nbk partials in block order,
// then the y update of Algorithm 2 as in k_t1_solve.
__global__ __launch_bounds__(kT) void k_t1_solve_p(const double *__restrict__ P, int nbk, int m,
                                                   double *__restrict__ y,
                                                   const double *__restrict__ y0,
                                                   double *__restrict__ ybar,
                                                   double *__restrict__ dy, IterScalars s,
                                                   int keep) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    if (i >= m) return;
    const double *Pi = P + (int64_t)i * nbk;
    double d0 = 0.0, d1 = 0.0, d2 = 0.0, d3 = 0.0;
    int k = lane;
    for (; k + 192 < nbk; k += 256) {
        d0 += Pi[k];
        d1 += Pi[k + 64];
        d2 += Pi[k + 128];
        d3 += Pi[k + 192];
    }
    for (; k < nbk; k += 64) d0 += Pi[k];
    const double d = wave_sum((d0 + d1) + (d2 + d3));
    if (lane != 0) return;
    const double yi = y[i];
    double yb = yi + d / s.sigma;
    if (i >= s.m1) yb = yb > 0.0 ? yb : 0.0;
    const double yr = s.rho == 2.0 ? 2.0 * yb - yi : s.rho * yb + (1.0 - s.rho) * yi;
    y[i] = s.hy0 * y0[i] + s.hy1 * yr;
    if (keep) {
        ybar[i] = yb;
        dy[i] = yi - yr;
    }
}

// parts[block] = sum over the block's columns j of (A~^T (va - vb))_j^2 (vb nullable);
// a fixed grid walks the columns in a fixed order
constexpr int kAtvBlocks = 1024;
__global__ __launch_bounds__(kT) void k_atv_sq(const int *__restrict__ rpt,
                                               const int *__restrict__ cit,
                                               const double *__restrict__ vat, int n,
                                               const double *__restrict__ va,
                                               const double *__restrict__ vb,
                                               double *__restrict__ parts) {
    __shared__ double red[kT / 64];
    double acc = 0.0;
    for (int j = blockIdx.x * kT + threadIdx.x; j < n; j += kAtvBlocks * kT) {
        double t = 0.0;
        for (int q = rpt[j]; q < rpt[j + 1]; ++q) {
            const int i = cit[q];
            t += vat[q] * (vb ? va[i] - vb[i] : va[i]);
        }
        acc += t * t;
    }
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kT / 64; ++w) s += red[w];
        parts[blockIdx.x] = s;
    }
}

__global__ __launch_bounds__(kT) void k_sum_parts(const double *__restrict__ parts, int np,
                                                  double *__restrict__ out) {
    __shared__ double red[kT / 64];
    double acc = 0.0;
    for (int k = threadIdx.x; k < np; k += kT) acc += parts[k];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int w = 0; w < kT / 64; ++w) s += red[w];
        *out = s;
    }
}

}  // namespace

size_t t1_parts_len() { return kAtvBlocks; }

int t1_padded_rows(int m) { return (m + kB - 1) / kB * kB; }

bool t1_lower_product(int m) {
    const size_t mp = (size_t)t1_padded_rows(m);
    return mp * mp * sizeof(double) > ((size_t)1 << 30);
}

size_t t1_partials_len(int m) {
    const size_t mp = (size_t)t1_padded_rows(m);
    return t1_lower_product(m) ? mp * (mp / kB) : 0;
}

hipError_t t1_build_inverse(const DevMat &A, const DevMat &T, int m, double *F, double *U,
                            double *V, double *Sb, double *diag0, double *diagd,
                            hipStream_t st) {
    const int mp = t1_padded_rows(m), nbk = mp / kB;
    const int ntiles = nbk * (nbk + 1) / 2;
    hipLaunchKernelGGL(k_gram, dim3(mp, (mp + kChunk - 1) / kChunk), dim3(64), 0, st, A.rp,
                       A.ci, static_cast<const double *>(A.va), T.rp, T.ci,
                       static_cast<const double *>(T.va), m, mp, F);
    hipLaunchKernelGGL(k_diag, dim3((m + 255) / 256), dim3(256), 0, st, F, m, mp, diag0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int p = 0; p < nbk; ++p) {
        hipLaunchKernelGGL(k_sweep_diag, dim3(1), dim3(kT), 0, st, F, mp, p * kB, Sb, diagd);
        if (nbk > 1)
            hipLaunchKernelGGL(k_sweep_panel, dim3(nbk), dim3(kT), 0, st, F, mp, p * kB, Sb,
                               U, V);
        hipLaunchKernelGGL(k_sweep_update, dim3(ntiles), dim3(kT), 0, st, F, mp, p * kB, Sb,
                           U, V);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_sweep_finish, dim3(ntiles), dim3(kT), 0, st, F, mp);
    return hipGetLastError();
}

hipError_t t1_row_step(const DevMat &A, const VecSet<double> &v, const IterScalars &s,
                       const double *G, double *r, double *P, int m, bool keep,
                       hipStream_t st) {
    const int nb = (m + kT / 64 - 1) / (kT / 64);
    hipError_t e = launch_t1_resid(A, v.xhat, v.bd, r, st);
    if (e != hipSuccess) return e;
    if (P) {
        const int nbk = t1_padded_rows(m) / kB;
        hipLaunchKernelGGL(k_t1_gr_tiles, dim3(nbk * (nbk + 1) / 2), dim3(kT), 0, st, G, r, m,
                           t1_padded_rows(m), nbk, P);
        hipLaunchKernelGGL(k_t1_solve_p, dim3(nb), dim3(kT), 0, st, P, nbk, m, v.y, v.y0,
                           v.ybar, v.dy, s, keep ? 1 : 0);
    } else {
        hipLaunchKernelGGL(k_t1_solve, dim3(nb), dim3(kT), 0, st, G, r, m, t1_padded_rows(m),
                           v.y, v.y0, v.ybar, v.dy, s, keep ? 1 : 0);
    }
    return hipGetLastError();
}

hipError_t t1_atv_sq(const DevMat &T, int n, const double *va, const double *vb, double *parts,
                     double *out, hipStream_t st) {
    hipLaunchKernelGGL(k_atv_sq, dim3(kAtvBlocks), dim3(kT), 0, st, T.rp, T.ci,
                       static_cast<const double *>(T.va), n, va, vb, parts);
    hipLaunchKernelGGL(k_sum_parts, dim3(1), dim3(kT), 0, st, parts, kAtvBlocks, out);
    return hipGetLastError();
}

}  // namespace hprlp
