/*
 * cabi_split.c -- drives libcgmi.so through its C ABI alone (no Python, no
 * torch): host-pointer vectors (cg_opts.vectors = CG_VECTORS_HOST), the row
 * split of Section 3.2 at GPU shares 0 (host only), 1/2 and 1, and the
 * memory modes of Section 3.4 (whole-segment and halo copies, mapped host
 * memory).  The matrix is the Dirichlet 7-point Laplacian on an N^3 grid
 * with b = A 1, so every solve must return x = 1 up to the tolerance, and
 * A 1 (integer sums) is exact in any summation order.
 *
 * Usage: cabi_split [N] [host_threads] [host].  With "host" only the
 * host-only handle runs (no HIP call at all, so also without a device), at
 * 1, 2 and host_threads threads.  Exit status 0 when every check passes.
 * Also the target of the sanitizer runs of the host runtime.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "../../include/cgmi.h"

static int failures = 0;

#define CHECK(cond, ...)                          \
    do {                                          \
        if (!(cond)) {                            \
            fprintf(stderr, "FAIL: " __VA_ARGS__); \
            fprintf(stderr, "\n");                \
            ++failures;                           \
        }                                         \
    } while (0)

int main(int argc, char **argv) {
    const int N = argc > 1 ? atoi(argv[1]) : 24;
    const int threads = argc > 2 ? atoi(argv[2]) : 4;
    const int host_only = argc > 3 && argv[3][0] == 'h';
    const int n = N * N * N;
    int32_t *rp = malloc(sizeof(int32_t) * (size_t)(n + 1));
    int32_t *ci = malloc(sizeof(int32_t) * (size_t)n * 7);
    double *va = malloc(sizeof(double) * (size_t)n * 7);
    double *b = malloc(sizeof(double) * (size_t)n), *x = malloc(sizeof(double) * (size_t)n);
    double *ones = malloc(sizeof(double) * (size_t)n), *y = malloc(sizeof(double) * (size_t)n);
    if (!rp || !ci || !va || !b || !x || !ones || !y) return 2;
    int64_t k = 0;
    rp[0] = 0;
    for (int i = 0; i < n; ++i) {
        const int ix = i % N, iy = (i / N) % N, iz = i / (N * N);
        const int nb[7] = {iz > 0 ? i - N * N : -1, iy > 0 ? i - N : -1, ix > 0 ? i - 1 : -1, i,
                           ix < N - 1 ? i + 1 : -1, iy < N - 1 ? i + N : -1, iz < N - 1 ? i + N * N : -1};
        double s = 0.0;
        for (int j = 0; j < 7; ++j) {
            if (nb[j] < 0) continue;
            ci[k] = nb[j];
            va[k] = nb[j] == i ? 6.0 : -1.0;
            s += va[k];
            ++k;
        }
        rp[i + 1] = (int32_t)k;
        b[i] = s;   /* (A 1)_i */
        ones[i] = 1.0;
    }
    struct { int32_t rb, re, exchange, threads; const char *name; } cases[] = {
        {0, 0, CG_EXCHANGE_WHOLE, 1, "host only, 1 thread"},
        {0, 0, CG_EXCHANGE_WHOLE, 2, "host only, 2 threads"},
        {0, 0, CG_EXCHANGE_WHOLE, 0, "host only"},
        {0, n / 2, CG_EXCHANGE_WHOLE, 0, "half, whole segments"},
        {0, n / 2, CG_EXCHANGE_HALO, 0, "half, halo"},
        {0, n / 2, CG_EXCHANGE_MAPPED, 0, "half, mapped p"},
        {n / 4, (3 * n) / 4, CG_EXCHANGE_HALO, 0, "middle half, halo"},
        {0, n, CG_EXCHANGE_WHOLE, 0, "GPU only"},
    };
    for (size_t c = 0; c < sizeof cases / sizeof cases[0]; ++c) {
        if (host_only && cases[c].re > cases[c].rb) continue;
        cg_handle *h = NULL;
        int rc = cg_create(n, k, rp, ci, va, cases[c].rb, cases[c].re, &h);
        CHECK(rc == CG_OK, "%s: cg_create %d (%s)", cases[c].name, rc, cg_last_error());
        if (rc != CG_OK) continue;
        cg_opts o;
        cg_default_opts(&o);
        o.vectors = CG_VECTORS_HOST;
        o.exchange = cases[c].exchange;
        o.host_threads = cases[c].threads ? cases[c].threads : threads;
        rc = cg_set_opts(h, &o);
        CHECK(rc == CG_OK, "%s: cg_set_opts %d (%s)", cases[c].name, rc, cg_last_error());
        rc = cg_spmv(h, ones, y);
        CHECK(rc == CG_OK, "%s: cg_spmv %d", cases[c].name, rc);
        int exact = 1;
        for (int i = 0; i < n; ++i) exact &= y[i] == b[i];
        CHECK(exact, "%s: A 1 differs from b", cases[c].name);
        for (int i = 0; i < n; ++i) x[i] = 0.0;
        cg_result r;
        rc = cg_solve(h, b, x, 1e-10, 10000, &r);
        double e = 0.0;
        for (int i = 0; i < n; ++i) e = fmax(e, fabs(x[i] - 1.0));
        CHECK(rc == CG_OK && r.converged && r.rel_res_true <= 1.01e-10, "%s: solve rc %d, rel. residual %.3e",
              cases[c].name, rc, r.rel_res_true);
        CHECK(e <= 1e-6, "%s: max |x - 1| = %.3e", cases[c].name, e);
        printf("%-22s rows gpu %8d cpu %8d: %4d iterations, true rel. residual %.2e, max |x-1| %.2e\n",
               cases[c].name, r.rows_gpu, r.rows_cpu, r.iterations, r.rel_res_true, e);
        cg_destroy(h);
    }
    free(rp); free(ci); free(va); free(b); free(x); free(ones); free(y);
    printf("%s\n", failures ? "FAILED" : "all checks passed");
    return failures ? 1 : 0;
}
