// The T1 = 0 variant of Section 3.2 (item 1) for LPs without inequality rows: the y-step
// is the exact minimiser of the augmented Lagrangian,
//     A~A~^T y_bar = (b~ - A~(x_bar + sigma (z_bar - c~))) / sigma        (eq. AATy=R),
// which, with the x-step, reads y_bar = y + G (b~ - A~ x_hat) / sigma, where G = (A~A~^T)^{-1}
// and x_hat = 2 x_bar - x.
//
// At create, G is formed once in the workspace: the dense Gram matrix A~A~^T (one workgroup
// per row, accumulated in LDS in a fixed order), its LDL^T factorisation (one launch per
// pivot), the inverse of the unit lower factor (one wavefront per column), and
// G = L^{-T} D^{-1} L^{-1} (an LDS-tiled product).  Every iteration then costs one residual
// pass over A~ and one dense matrix-vector product with G (m^2 FP64 reads, HBM-bound), with
// the y epilogue of Algorithm 2 fused into it.  The checks need ||A~^T v||^2 (M of eq.
// def:M with T1 = 0, and eq. sigma_T1=0), from one pass over A~^T.
#include <hip/hip_runtime.h>

#include <cstdint>

#include "hprlp_internal.h"

namespace hprlp {
namespace {

constexpr int kT = 256;  // threads per block of the row-wise kernels (4 wavefronts)
constexpr int kTile = 16;

__device__ __forceinline__ double wave_sum(double v) {
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// F[i][k] = <row i of A~, row k of A~> for all k: workgroup i scatters, for each nonzero
// (i, j) of its row in storage order, a_ij * A~^T row j into an LDS row of length m.
__global__ __launch_bounds__(kT) void k_gram(const int *__restrict__ rp,
                                             const int *__restrict__ ci,
                                             const double *__restrict__ va,
                                             const int *__restrict__ rpt,
                                             const int *__restrict__ cit,
                                             const double *__restrict__ vat, int m,
                                             double *__restrict__ F) {
    extern __shared__ double acc[];
    const int i = blockIdx.x;
    for (int k = threadIdx.x; k < m; k += kT) acc[k] = 0.0;
    __syncthreads();
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        const int j = ci[p];
        const double a = va[p];
        // the rows k of column j are distinct: no two threads touch the same entry
        for (int q = rpt[j] + threadIdx.x; q < rpt[j + 1]; q += kT) acc[cit[q]] += a * vat[q];
        __syncthreads();
    }
    for (int k = threadIdx.x; k < m; k += kT) F[(int64_t)i * m + k] = acc[k];
}

__global__ void k_diag(const double *__restrict__ F, int m, double *__restrict__ d) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < m) d[i] = F[(int64_t)i * m + i];
}

// One elimination step of LDL^T on the lower triangle: F_ij -= F_ik F_jk / F_kk for
// k < j <= i < m, a 64 x 64 tile per 16 x 16 block (4 x 4 entries per thread, rows and
// columns strided by 16).  Column k is read, never written, in this step.
constexpr int kLdl = 64;
__global__ void k_ldl_step(double *__restrict__ F, int m, int k) {
    const int i0 = k + 1 + blockIdx.y * kLdl, j0 = k + 1 + blockIdx.x * kLdl;
    if (j0 > i0 + kLdl - 1) return;  // tile above the diagonal
    const double fkk = F[(int64_t)k * m + k];
    double fi[4], fj[4];
    for (int a = 0; a < 4; ++a) {
        const int i = i0 + threadIdx.y + 16 * a, j = j0 + threadIdx.x + 16 * a;
        fi[a] = i < m ? F[(int64_t)i * m + k] : 0.0;
        fj[a] = j < m ? F[(int64_t)j * m + k] : 0.0;
    }
    for (int a = 0; a < 4; ++a) {
        const int i = i0 + threadIdx.y + 16 * a;
        if (i >= m) break;
        for (int b = 0; b < 4; ++b) {
            const int j = j0 + threadIdx.x + 16 * b;
            if (j <= i) F[(int64_t)i * m + j] -= fi[a] * fj[b] / fkk;
        }
    }
}

// unit lower factor in place: F_ik <- F_ik / F_kk for i > k (the diagonal keeps D)
__global__ void k_unit_lower(double *__restrict__ F, int m) {
    const int i = blockIdx.y * kTile + threadIdx.y, k = blockIdx.x * kTile + threadIdx.x;
    if (i < m && k < i) F[(int64_t)i * m + k] = F[(int64_t)i * m + k] / F[(int64_t)k * m + k];
}

// LT[c][i] = (L^{-1})_{ic}: column c of the inverse of the unit lower factor, by forward
// substitution (rows i > c in order), one wavefront per column, the column kept in LDS.
__global__ __launch_bounds__(64) void k_linv(const double *__restrict__ F, int m,
                                             double *__restrict__ LT) {
    extern __shared__ double col[];
    const int c = blockIdx.x, lane = threadIdx.x;
    for (int k = lane; k < m; k += 64) col[k] = k == c ? 1.0 : 0.0;
    __syncthreads();
    for (int i = c + 1; i < m; ++i) {
        const double *Li = F + (int64_t)i * m;
        double acc = 0.0;
        for (int k = c + lane; k < i; k += 64) acc += Li[k] * col[k];
        acc = wave_sum(acc);
        if (lane == 0) col[i] = -acc;
        __syncthreads();
    }
    for (int k = lane; k < m; k += 64) LT[(int64_t)c * m + k] = col[k];
}

// G[a][b] = sum_k LT[a][k] LT[b][k] / d_k  (= (L^{-T} D^{-1} L^{-1})_{ab}), in 16 x 16 tiles
// with the k range staged through LDS in steps of 16, in increasing k.
__global__ void k_gram_inverse(const double *__restrict__ LT, const double *__restrict__ F,
                               int m, double *__restrict__ G) {
    __shared__ double ta[kTile][kTile + 1], tb[kTile][kTile + 1];
    const int a0 = blockIdx.y * kTile, b0 = blockIdx.x * kTile;
    const int ty = threadIdx.y, tx = threadIdx.x;
    const int a = a0 + ty, b = b0 + tx;
    const int kstart = (a0 > b0 ? a0 : b0);  // LT[r][k] = 0 for k < r
    double acc = 0.0;
    for (int k0 = kstart - kstart % kTile; k0 < m; k0 += kTile) {
        const int k = k0 + tx;
        const int ra = a0 + ty, rb = b0 + ty;
        ta[ty][tx] = (ra < m && k < m) ? LT[(int64_t)ra * m + k] : 0.0;
        tb[ty][tx] = (rb < m && k < m) ? LT[(int64_t)rb * m + k] / F[(int64_t)k * m + k] : 0.0;
        __syncthreads();
        for (int q = 0; q < kTile; ++q) acc += ta[ty][q] * tb[tx][q];
        __syncthreads();
    }
    if (a < m && b < m) G[(int64_t)a * m + b] = acc;
}

// r = b~ - A~ x_hat (one wavefront per row)
__global__ __launch_bounds__(kT) void k_t1_resid(const int *__restrict__ rp,
                                                 const int *__restrict__ ci,
                                                 const double *__restrict__ va,
                                                 const double *__restrict__ xh,
                                                 const double *__restrict__ bd, int m,
                                                 double *__restrict__ r) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    if (i >= m) return;
    double s = 0.0;
    for (int p = rp[i] + lane; p < rp[i + 1]; p += 64) s += va[p] * xh[ci[p]];
    s = wave_sum(s);
    if (lane == 0) r[i] = bd[i] - s;
}

// y-step with T1 = 0 and the rest of Algorithm 2's y update, one wavefront per row:
// y_bar = y + (G r)_i / sigma; relaxed point rho y_bar + (1 - rho) y; Halpern average.
__global__ __launch_bounds__(kT) void k_t1_solve(const double *__restrict__ G,
                                                 const double *__restrict__ r, int m,
                                                 double *__restrict__ y,
                                                 const double *__restrict__ y0,
                                                 double *__restrict__ ybar,
                                                 double *__restrict__ dy, IterScalars s,
                                                 int keep) {
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * (kT / 64) + (threadIdx.x >> 6);
    if (i >= m) return;
    const double *Gi = G + (int64_t)i * m;
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

hipError_t t1_build_inverse(const DevMat &A, const DevMat &T, int m, double *F, double *LT,
                            double *G, double *diag0, double *diagd, hipStream_t st) {
    const size_t lds = sizeof(double) * (size_t)m;
    hipLaunchKernelGGL(k_gram, dim3(m), dim3(kT), lds, st, A.rp, A.ci,
                       static_cast<const double *>(A.va), T.rp, T.ci,
                       static_cast<const double *>(T.va), m, F);
    hipLaunchKernelGGL(k_diag, dim3((m + 255) / 256), dim3(256), 0, st, F, m, diag0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    for (int k = 0; k + 1 < m; ++k) {
        const int nt = (m - k - 1 + kLdl - 1) / kLdl;
        hipLaunchKernelGGL(k_ldl_step, dim3(nt, nt), dim3(16, 16), 0, st, F, m, k);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    hipLaunchKernelGGL(k_diag, dim3((m + 255) / 256), dim3(256), 0, st, F, m, diagd);
    const int nt = (m + kTile - 1) / kTile;
    hipLaunchKernelGGL(k_unit_lower, dim3(nt, nt), dim3(kTile, kTile), 0, st, F, m);
    hipLaunchKernelGGL(k_linv, dim3(m), dim3(64), lds, st, F, m, LT);
    hipLaunchKernelGGL(k_gram_inverse, dim3(nt, nt), dim3(kTile, kTile), 0, st, LT, F, m, G);
    return hipGetLastError();
}

hipError_t t1_row_step(const DevMat &A, const VecSet<double> &v, const IterScalars &s,
                       const double *G, double *r, int m, bool keep, hipStream_t st) {
    const int nb = (m + kT / 64 - 1) / (kT / 64);
    hipLaunchKernelGGL(k_t1_resid, dim3(nb), dim3(kT), 0, st, A.rp, A.ci,
                       static_cast<const double *>(A.va), v.xhat, v.bd, m, r);
    hipLaunchKernelGGL(k_t1_solve, dim3(nb), dim3(kT), 0, st, G, r, m, v.y, v.y0, v.ybar,
                       v.dy, s, keep ? 1 : 0);
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
