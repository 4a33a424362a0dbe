/* Drives the CPU oracle (oracle/oracle.c) under AddressSanitizer and
 * UndefinedBehaviorSanitizer: SpMV, block SpMV, CG and the true relative
 * residual on a 27-point stencil built here, including an empty matrix and
 * an empty row.  Exit status 0 when every check holds (test infrastructure). */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int oracle_threads(void);
void oracle_set_threads(int t);
void oracle_spmv(int64_t n_rows, const int64_t *row_ptr, const int32_t *col, const double *val, const double *x,
                 double *y);
void oracle_spmv_block(int64_t n_rows, const int64_t *row_ptr, const int32_t *col, const double *val, int32_t nrhs,
                       const double *X, int64_t ldx, double *Y, int64_t ldy);
double oracle_relres(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val, const double *b,
                     const double *x);
int oracle_cg(int64_t n, const int64_t *row_ptr, const int32_t *col, const double *val, const double *b, double *x,
              double rtol, int32_t max_iter, int32_t *iters, double *relres_rec);

#define CHECK(c)                                                    \
    do {                                                            \
        if (!(c)) {                                                 \
            fprintf(stderr, "check failed: %s (line %d)\n", #c, __LINE__); \
            return 1;                                               \
        }                                                           \
    } while (0)

int main(void) {
    const int nx = 6, ny = 5, nz = 4, n = nx * ny * nz;
    int64_t *rp = malloc(sizeof(int64_t) * (n + 1));
    int32_t *col = malloc(sizeof(int32_t) * n * 27);
    double *val = malloc(sizeof(double) * n * 27);
    int64_t k = 0;
    rp[0] = 0;
    for (int i = 0; i < n; ++i) {
        const int ix = i % nx, iy = (i / nx) % ny, iz = i / (nx * ny);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    const int jx = ix + dx, jy = iy + dy, jz = iz + dz;
                    if (jx < 0 || jx >= nx || jy < 0 || jy >= ny || jz < 0 || jz >= nz) continue;
                    col[k] = jx + nx * (jy + ny * jz);
                    val[k] = (dx == 0 && dy == 0 && dz == 0) ? 26.0 : -1.0;
                    ++k;
                }
        rp[i + 1] = k;
    }
    double *one = malloc(sizeof(double) * n), *b = malloc(sizeof(double) * n), *x = malloc(sizeof(double) * n);
    for (int i = 0; i < n; ++i) one[i] = 1.0;
    oracle_spmv(n, rp, col, val, one, b);
    for (int i = 0; i < n; ++i) CHECK(b[i] == 26.0 - (double)(rp[i + 1] - rp[i] - 1));
    /* block SpMV with a leading dimension above nrhs */
    double *X = malloc(sizeof(double) * n * 5), *Y = malloc(sizeof(double) * n * 5);
    for (int i = 0; i < n * 5; ++i) X[i] = (double)((i * 37) % 11) - 5.0;
    oracle_spmv_block(n, rp, col, val, 3, X, 5, Y, 5);
    for (int r = 0; r < 3; ++r) {
        for (int i = 0; i < n; ++i) x[i] = X[(int64_t)i * 5 + r];
        oracle_spmv(n, rp, col, val, x, one);
        for (int i = 0; i < n; ++i) CHECK(one[i] == Y[(int64_t)i * 5 + r]);
    }
    for (int i = 0; i < n; ++i) one[i] = 1.0;
    int32_t iters = 0;
    double rec = 0.0;
    const int t = oracle_threads();
    CHECK(t >= 1);
    oracle_set_threads(1);
    const int st = oracle_cg(n, rp, col, val, b, x, 1e-10, 1000, &iters, &rec);
    oracle_set_threads(t);
    CHECK(st == 0 && iters > 0 && rec <= 1e-10);
    CHECK(oracle_relres(n, rp, col, val, b, x) <= 1e-10);
    for (int i = 0; i < n; ++i) CHECK(fabs(x[i] - 1.0) < 1e-8);
    CHECK(oracle_cg(n, rp, col, val, b, x, 1e-10, 3, &iters, &rec) == -7 && iters == 3);
    /* empty matrix; a matrix whose only row is empty */
    int64_t rp0[2] = {0, 0};
    oracle_spmv(0, rp0, col, val, one, b);
    CHECK(oracle_cg(0, rp0, col, val, b, x, 1e-10, 10, &iters, &rec) == 0);
    b[0] = 7.0;
    oracle_spmv(1, rp0, col, val, one, b);
    CHECK(b[0] == 0.0);
    free(rp); free(col); free(val); free(one); free(b); free(x); free(X); free(Y);
    puts("oracle sanitizer driver: ok");
    return 0;
}
