/*
 * CPU oracle for compressed SpMV and CG -- TEST INFRASTRUCTURE ONLY.
 *
 * Only the test-suite, the smoke check and the benchmark's CPU-baseline leg
 * may load this library.  It shares no code with the GPU library.
 *
 * Everything here is the plain definition, in FP64, compiled with
 * -ffp-contract=off so that every product is rounded before it is added:
 *
 *   oracle_spmv        y = A x  (Eq. 1, Section I), CSR, each row summed in
 *                      ascending column order starting from +0.0.
 *   oracle_spmv_block  Y = A X  for row-interleaved X (element (j, r) at
 *                      X[j*ldx + r]); the single-vector definition per column.
 *   oracle_cg          unpreconditioned conjugate gradients (the CG part of the
 *                      iteration in Table I, Section III-C: DotProduct, Waxpby,
 *                      SpMV), textbook Hestenes-Stiefel form (Saad, "Iterative
 *                      Methods for Sparse Linear Systems", 2nd ed., Alg. 6.18).
 *
 * Rows are independent in the SpMV, so it runs rows in parallel with OpenMP;
 * that does not change any result bit.  Dot products are serial, in index
 * order, so CG is bit-reproducible for any thread count.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

int oracle_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

void oracle_set_threads(int t) {
#ifdef _OPENMP
    if (t > 0) omp_set_num_threads(t);
#else
    (void)t;
#endif
}

/* y_i = sum_k val[k] * x[col[k]], k over row i in stored (ascending column) order. */
void oracle_spmv(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                 const double *val, const double *x, double *y) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_rows; ++i) {
        double s = 0.0;
        for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
            double prod = val[k] * x[col[k]];
            s = s + prod;
        }
        y[i] = s;
    }
}

/* Y = A X, row-interleaved: X(j, r) = X[j*ldx + r], Y(i, r) = Y[i*ldy + r]. */
void oracle_spmv_block(int64_t n_rows, const int64_t *row_ptr, const int32_t *col,
                       const double *val, int32_t nrhs, const double *X, int64_t ldx,
                       double *Y, int64_t ldy) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_rows; ++i) {
        for (int32_t r = 0; r < nrhs; ++r) {
            double s = 0.0;
            for (int64_t k = row_ptr[i]; k < row_ptr[i + 1]; ++k) {
                double prod = val[k] * X[(int64_t)col[k] * ldx + r];
                s = s + prod;
            }
            Y[i * ldy + r] = s;
        }
    }
}

static double dot_serial(int64_t n, const double *a, const double *b) {
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double prod = a[i] * b[i];
        s = s + prod;
    }
    return s;
}

/* ||b - A x||_2 / ||b||_2 (returns ||b - A x||_2 when b == 0). */
double oracle_relres(int64_t n, const int64_t *row_ptr, const int32_t *col,
                     const double *val, const double *b, const double *x) {
    double *ax = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!ax) return NAN;
    oracle_spmv(n, row_ptr, col, val, x, ax);
    double rr = 0.0, bb = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double d = b[i] - ax[i];
        rr = rr + d * d;
        bb = bb + b[i] * b[i];
    }
    free(ax);
    return bb > 0.0 ? sqrt(rr) / sqrt(bb) : sqrt(rr);
}

/*
 * Unpreconditioned CG from x0 = 0:
 *   r = b, p = r, rho = r.r
 *   loop:  q = A p;  sigma = p.q  (sigma <= 0 or non-finite -> not SPD, -6)
 *          alpha = rho / sigma;  x += alpha p;  r -= alpha q
 *          rho' = r.r;  stop when sqrt(rho') <= rtol * ||b||
 *          beta = rho' / rho;  p = r + beta p
 * Returns 0 on convergence, -6 on breakdown, -7 when max_iter SpMVs were done
 * without convergence.  *iters = number of SpMVs in the loop; *relres_rec =
 * sqrt(rho') / ||b|| at exit.  x receives the last iterate.
 */
int oracle_cg(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val,
              const double *b, double *x, double rtol, int32_t max_iter,
              int32_t *iters, double *relres_rec) {
    double *r = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    double *q = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!r || !p || !q) {
        free(r); free(p); free(q);
        return -2;
    }
    for (int64_t i = 0; i < n; ++i) {
        x[i] = 0.0;
        r[i] = b[i];
        p[i] = b[i];
    }
    double rho = dot_serial(n, r, r);
    double bnorm = sqrt(rho);
    int status = -7;
    int32_t k = 0;
    if (bnorm == 0.0) {
        status = 0;
        *iters = 0;
        *relres_rec = 0.0;
        free(r); free(p); free(q);
        return status;
    }
    double rel = 1.0;
    while (k < max_iter) {
        oracle_spmv(n, row_ptr, col, val, p, q);
        ++k;
        double sigma = dot_serial(n, p, q);
        if (!(sigma > 0.0) || !isfinite(sigma)) {
            status = -6;
            break;
        }
        double alpha = rho / sigma;
        for (int64_t i = 0; i < n; ++i) {
            x[i] = x[i] + alpha * p[i];
            r[i] = r[i] - alpha * q[i];
        }
        double rho_new = dot_serial(n, r, r);
        rel = sqrt(rho_new) / bnorm;
        if (sqrt(rho_new) <= rtol * bnorm) {
            status = 0;
            rho = rho_new;
            break;
        }
        double beta = rho_new / rho;
        for (int64_t i = 0; i < n; ++i) p[i] = r[i] + beta * p[i];
        rho = rho_new;
    }
    *iters = k;
    *relres_rec = rel;
    free(r); free(p); free(q);
    return status;
}
