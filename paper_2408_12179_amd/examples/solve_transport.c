/* Solving one LP through the C ABI alone (no Python, no torch): a 2 x 3 transportation
 * problem, min <c, x> s.t. supply rows sum_j x_ij = s_i (equalities), demand rows
 * sum_i x_ij >= d_j (inequalities), x >= 0.  The caller owns the device workspace.
 *
 * Build (plain C): gcc -O2 -D__HIP_PLATFORM_AMD__ -I/opt/rocm/include -I<repo>/include
 *   solve_transport.c -L<dir of libhprlp.so> -lhprlp -L/opt/rocm/lib -lamdhip64 -lm
 * Prints the status, the iteration count and the primal objective. */
#include <hip/hip_runtime_api.h>
#include <math.h>
#include <stdio.h>

#include "hprlp.h"

int main(void) {
    const int64_t m1 = 2, m2 = 3, n = 6;
    const int64_t rowptr[] = {0, 3, 6, 8, 10, 12};
    const int32_t colidx[] = {0, 1, 2, 3, 4, 5, 0, 3, 1, 4, 2, 5};
    const double val[] = {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1};
    const double b[] = {20, 30, 10, 25, 15};          /* supplies, then demands */
    const double c[] = {4, 6, 9, 5, 3, 8};            /* cost of x_ij at column 3 i + j */
    const double l[] = {0, 0, 0, 0, 0, 0};
    const double u[] = {INFINITY, INFINITY, INFINITY, INFINITY, INFINITY, INFINITY};

    hprlp_options opt;
    hprlp_default_options(&opt);
    size_t bytes = 0;
    if (hprlp_workspace_bytes(m1, m2, n, rowptr[m1 + m2], &opt, &bytes) != HPRLP_OK) {
        fprintf(stderr, "workspace_bytes: %s\n", hprlp_last_error(NULL));
        return 1;
    }
    void *ws = NULL;
    if (hipMalloc(&ws, bytes) != hipSuccess) {
        fprintf(stderr, "hipMalloc of %zu bytes failed\n", bytes);
        return 1;
    }
    hprlp_handle *h = NULL;
    int rc = hprlp_create(&h, m1, m2, n, rowptr, colidx, val, b, c, l, u, &opt, ws, bytes, NULL);
    if (rc != HPRLP_OK) {
        fprintf(stderr, "create: %d %s\n", rc, hprlp_last_error(NULL));
        hipFree(ws);
        return 1;
    }
    double x[6], y[5], z[6];
    int status = 0;
    rc = hprlp_solve(h, x, y, z, &status);
    hprlp_stats_t st;
    if (rc == HPRLP_OK) rc = hprlp_stats(h, &st);
    if (rc != HPRLP_OK) {
        fprintf(stderr, "solve: %d %s\n", rc, hprlp_last_error(h));
    } else {
        printf("status %d iters %lld pobj %.12g\n", status, st.iters, st.pobj);
        printf("x %.6g %.6g %.6g %.6g %.6g %.6g\n", x[0], x[1], x[2], x[3], x[4], x[5]);
    }
    hprlp_destroy(h);
    hipFree(ws);
    return rc == HPRLP_OK && status == HPRLP_OPTIMAL ? 0 : 2;
}
