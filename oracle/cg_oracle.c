/*
 * cg_oracle.c -- plain CPU oracle for the sparse conjugate-gradient hot path.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, calls or
 * includes this file; only the tests, the smoke check and the CPU baseline of
 * the benchmark use it.  It shares no code, header, table or helper with the
 * GPU path.
 *
 * Everything here is the obvious textbook loop, in float64 unless a routine
 * says otherwise, with no blocking, fusion or reordering:
 *   - CSR SpMV (q_i = sum_j A_ij p_j, Section 3.1): each row summed left to
 *     right in CSR order, product rounded then added (built with
 *     -ffp-contract=off).  Rows may be spread over threads; a row's sum order
 *     never changes, so results do not depend on the thread count.
 *   - dot products: one left-to-right sum.
 *   - CG: Algorithm 1 (Section 3.1) step for step, with the stop test read as
 *     relative, sqrt(rho) < tol * ||b||_2, at the top of each iteration.
 *   - PCG with M^{-1} = G^T G (factored sparse approximate inverse).
 *   - mixed precision: float32 inner CG with float64 reliable updates
 *     (true residual b - A x, its norm and the solution x kept in float64).
 *
 * Return codes match the library's: 0 converged, 1 iteration limit reached,
 * -1 invalid argument, -4 breakdown (p^T q <= 0 or not finite).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_MAXIT 1
#define ORC_EINVAL (-1)
#define ORC_ENOMEM (-2)
#define ORC_EBREAKDOWN (-4)

/* y = A x over rows [0, n) of a CSR matrix with ncols columns (Section 3.1). */
void oracle_spmv(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                 const double *x, double *y)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        double s = 0.0;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            s += v[k] * x[ci[k]];
        y[i] = s;
    }
}

/* float32 SpMV on float32 values and vector. */
void oracle_spmv_f32(int32_t n, const int32_t *rp, const int32_t *ci, const float *v,
                     const float *x, float *y)
{
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i) {
        float s = 0.0f;
        for (int32_t k = rp[i]; k < rp[i + 1]; ++k)
            s += v[k] * x[ci[k]];
        y[i] = s;
    }
}

double oracle_dot(int64_t n, const double *x, const double *y)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += x[i] * y[i];
    return s;
}

/* float32 vectors, products and sums formed in float64. */
static double dot_f32(int64_t n, const float *x, const float *y)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i)
        s += (double)x[i] * (double)y[i];
    return s;
}

/* r = b - A x */
static void residual(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                     const double *b, const double *x, double *r)
{
    oracle_spmv(n, rp, ci, v, x, r);
#pragma omp parallel for schedule(static)
    for (int32_t i = 0; i < n; ++i)
        r[i] = b[i] - r[i];
}

static int bad_rho(double d) { return !(d > 0.0) || !isfinite(d); }

/*
 * Unpreconditioned CG, Algorithm 1 (Section 3.1):
 *   r = b - A x, p = r, rho = r^T r
 *   for k = 0 .. maxit-1:
 *     stop if sqrt(rho) < tol*||b||  (or rho == 0)
 *     q = A p; alpha = rho / p^T q; x += alpha p; r -= alpha q
 *     rho_old = rho; rho = r^T r; beta = rho / rho_old; p = r + beta p
 * After the loop the true residual ||b - A x|| / ||b|| is recomputed
 * (Section 3.1, verification after each solve).
 *
 * iters[0]   : number of iterations performed (SpMVs inside the loop)
 * rho_hist   : optional, rho before iteration k for k = 0..iters (maxit+1 slots)
 * relres[0]  : sqrt(rho)/||b|| at exit; relres[1]: ||b - A x|| / ||b||
 */
int oracle_cg(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
              const double *b, double *x, double tol, int32_t maxit,
              int32_t *iters, double *rho_hist, double *relres)
{
    if (n < 0 || maxit < 0 || !(tol >= 0.0))
        return ORC_EINVAL;
    iters[0] = 0;
    relres[0] = relres[1] = 0.0;
    if (n == 0)
        return ORC_OK;
    double *r = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n);
    double *q = malloc(sizeof(double) * (size_t)n);
    if (!r || !p || !q) {
        free(r); free(p); free(q);
        return ORC_ENOMEM;
    }
    double bnorm = sqrt(oracle_dot(n, b, b));
    int status = ORC_MAXIT;
    if (bnorm == 0.0) {           /* A x = 0 has the solution x = 0 */
        memset(x, 0, sizeof(double) * (size_t)n);
        free(r); free(p); free(q);
        return ORC_OK;
    }
    residual(n, rp, ci, v, b, x, r);
    memcpy(p, r, sizeof(double) * (size_t)n);
    double rho = oracle_dot(n, r, r);
    if (rho_hist)
        rho_hist[0] = rho;
    int32_t k = 0;
    for (k = 0; k < maxit; ++k) {
        if (sqrt(rho) < tol * bnorm || rho == 0.0) {
            status = ORC_OK;
            break;
        }
        oracle_spmv(n, rp, ci, v, p, q);
        double pq = oracle_dot(n, p, q);
        if (bad_rho(pq)) {
            status = ORC_EBREAKDOWN;
            break;
        }
        double alpha = rho / pq;
        for (int32_t i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * p[i];
            r[i] = r[i] - alpha * q[i];
        }
        double rho_old = rho;
        rho = oracle_dot(n, r, r);
        double beta = rho / rho_old;
        for (int32_t i = 0; i < n; ++i)
            p[i] = r[i] + beta * p[i];
        if (rho_hist)
            rho_hist[k + 1] = rho;
    }
    if (status == ORC_MAXIT && (sqrt(rho) < tol * bnorm || rho == 0.0))
        status = ORC_OK;
    iters[0] = k;
    relres[0] = sqrt(rho) / bnorm;
    residual(n, rp, ci, v, b, x, r);
    relres[1] = sqrt(oracle_dot(n, r, r)) / bnorm;
    free(r); free(p); free(q);
    return status;
}

/*
 * Preconditioned CG with M^{-1} = G^T G, applied as z = G^T (G r) with G and
 * G^T given as explicit CSR matrices.  The stop test is on the unpreconditioned
 * residual, sqrt(r^T r) < tol*||b||, so that plain and preconditioned solves
 * meet the same criterion.  With G = I every step coincides with oracle_cg.
 */
int oracle_pcg(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
               const int32_t *grp, const int32_t *gci, const double *gv,
               const int32_t *trp, const int32_t *tci, const double *tv,
               const double *b, double *x, double tol, int32_t maxit,
               int32_t *iters, double *relres)
{
    if (n < 0 || maxit < 0 || !(tol >= 0.0))
        return ORC_EINVAL;
    iters[0] = 0;
    relres[0] = relres[1] = 0.0;
    if (n == 0)
        return ORC_OK;
    double *r = malloc(sizeof(double) * (size_t)n);
    double *p = malloc(sizeof(double) * (size_t)n);
    double *q = malloc(sizeof(double) * (size_t)n);
    double *t = malloc(sizeof(double) * (size_t)n);
    double *z = malloc(sizeof(double) * (size_t)n);
    if (!r || !p || !q || !t || !z) {
        free(r); free(p); free(q); free(t); free(z);
        return ORC_ENOMEM;
    }
    double bnorm = sqrt(oracle_dot(n, b, b));
    int status = ORC_MAXIT;
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        free(r); free(p); free(q); free(t); free(z);
        return ORC_OK;
    }
    residual(n, rp, ci, v, b, x, r);
    oracle_spmv(n, grp, gci, gv, r, t);
    oracle_spmv(n, trp, tci, tv, t, z);
    memcpy(p, z, sizeof(double) * (size_t)n);
    double rho = oracle_dot(n, r, z);
    double rr = oracle_dot(n, r, r);
    int32_t k = 0;
    for (k = 0; k < maxit; ++k) {
        if (sqrt(rr) < tol * bnorm || rr == 0.0) {
            status = ORC_OK;
            break;
        }
        oracle_spmv(n, rp, ci, v, p, q);
        double pq = oracle_dot(n, p, q);
        if (bad_rho(pq)) {
            status = ORC_EBREAKDOWN;
            break;
        }
        double alpha = rho / pq;
        for (int32_t i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * p[i];
            r[i] = r[i] - alpha * q[i];
        }
        oracle_spmv(n, grp, gci, gv, r, t);
        oracle_spmv(n, trp, tci, tv, t, z);
        double rho_old = rho;
        rho = oracle_dot(n, r, z);
        rr = oracle_dot(n, r, r);
        if (bad_rho(rho) && rr != 0.0) {
            status = ORC_EBREAKDOWN;
            ++k;
            break;
        }
        double beta = rho / rho_old;
        for (int32_t i = 0; i < n; ++i)
            p[i] = z[i] + beta * p[i];
    }
    if (status == ORC_MAXIT && (sqrt(rr) < tol * bnorm || rr == 0.0))
        status = ORC_OK;
    iters[0] = k;
    relres[0] = sqrt(rr) / bnorm;
    residual(n, rp, ci, v, b, x, r);
    relres[1] = sqrt(oracle_dot(n, r, r)) / bnorm;
    free(r); free(p); free(q); free(t); free(z);
    return status;
}

/*
 * Mixed precision: float32 inner CG with float64 refinement by reliable
 * updates.  The matrix values and the inner vectors r, p, q are float32; the
 * SpMV and the vector updates of r and p run in float32; dot products are
 * accumulated in float64.  The solution x is float64 and is updated in
 * float64 every iteration (x += alpha p).  Whenever the float32 recurrence
 * residual has dropped by the factor delta since the last refinement, or
 * meets the tolerance, the true residual b - A x is recomputed in float64,
 * its norm taken in float64, and the float32 residual replaced by it.  The
 * solve ends when that float64 true residual meets tol*||b||.
 *
 *   counts[0] : float32 inner iterations;  counts[1] : float64 residuals formed
 *   relres[0] : last float64 true residual / ||b||; relres[1] : same, recomputed
 */
int oracle_cg_mixed(int32_t n, const int32_t *rp, const int32_t *ci, const double *v,
                    const double *b, double *x, double tol, int32_t maxit, double delta,
                    int32_t *counts, double *relres)
{
    if (n < 0 || maxit < 0 || !(tol >= 0.0) || !(delta > 0.0 && delta < 1.0))
        return ORC_EINVAL;
    counts[0] = counts[1] = 0;
    relres[0] = relres[1] = 0.0;
    if (n == 0)
        return ORC_OK;
    int64_t nnz = rp[n];
    float *v32 = malloc(sizeof(float) * (size_t)(nnz > 0 ? nnz : 1));
    float *r = malloc(sizeof(float) * (size_t)n);
    float *p = malloc(sizeof(float) * (size_t)n);
    float *q = malloc(sizeof(float) * (size_t)n);
    double *r64 = malloc(sizeof(double) * (size_t)n);
    if (!v32 || !r || !p || !q || !r64) {
        free(v32); free(r); free(p); free(q); free(r64);
        return ORC_ENOMEM;
    }
    for (int64_t k = 0; k < nnz; ++k)
        v32[k] = (float)v[k];
    double bnorm = sqrt(oracle_dot(n, b, b));
    if (bnorm == 0.0) {
        memset(x, 0, sizeof(double) * (size_t)n);
        free(v32); free(r); free(p); free(q); free(r64);
        return ORC_OK;
    }
    int status = ORC_MAXIT;
    residual(n, rp, ci, v, b, x, r64);
    counts[1] = 1;
    double true_norm = sqrt(oracle_dot(n, r64, r64));
    for (int32_t i = 0; i < n; ++i)
        r[i] = (float)r64[i];
    memcpy(p, r, sizeof(float) * (size_t)n);
    double rho = dot_f32(n, r, r);
    double rmax = sqrt(rho);
    int32_t k = 0;
    if (true_norm < tol * bnorm || true_norm == 0.0)
        status = ORC_OK;
    else {
        for (k = 0; k < maxit;) {
            oracle_spmv_f32(n, rp, ci, v32, p, q);
            double pq = dot_f32(n, p, q);
            if (bad_rho(pq)) {
                status = ORC_EBREAKDOWN;
                break;
            }
            double alpha = rho / pq;
            float alpha32 = (float)alpha;
            for (int32_t i = 0; i < n; ++i) {
                x[i] = x[i] + alpha * (double)p[i];
                r[i] = r[i] - alpha32 * q[i];
            }
            ++k;
            double rho_new = dot_f32(n, r, r);
            if (sqrt(rho_new) < delta * rmax || sqrt(rho_new) < tol * bnorm) {
                /* float64 refinement: true residual, its norm, fresh float32 residual */
                residual(n, rp, ci, v, b, x, r64);
                counts[1] += 1;
                true_norm = sqrt(oracle_dot(n, r64, r64));
                if (true_norm < tol * bnorm || true_norm == 0.0) {
                    status = ORC_OK;
                    break;
                }
                for (int32_t i = 0; i < n; ++i)
                    r[i] = (float)r64[i];
                rho_new = dot_f32(n, r, r);
                rmax = sqrt(rho_new);
            }
            float beta32 = (float)(rho_new / rho);
            rho = rho_new;
            for (int32_t i = 0; i < n; ++i)
                p[i] = r[i] + beta32 * p[i];
        }
    }
    counts[0] = k;
    relres[0] = true_norm / bnorm;
    residual(n, rp, ci, v, b, x, r64);
    relres[1] = sqrt(oracle_dot(n, r64, r64)) / bnorm;
    free(v32); free(r); free(p); free(q); free(r64);
    return status;
}

/* Thread control for the row loops (dot products are always one serial sum). */
#include <omp.h>
void oracle_set_threads(int32_t t) { if (t > 0) omp_set_num_threads(t); }
int32_t oracle_max_threads(void) { return (int32_t)omp_get_max_threads(); }
