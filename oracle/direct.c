/*
 * ORACLE -- test infrastructure only.  Only tests/, the smoke entry and the
 * benchmark's CPU-baseline leg may load this code; the GPU library never does.
 *
 * Plain FP64 direct kernel summation, the definition the paper's fast
 * summation approximates (Sec. 4, eq. for (W~v)_i, with the self term removed
 * as in the W = W~ - K(0) I identity; Sec. 2 for the zero diagonal):
 *
 *     y_i = sum_{j != i} K(x_i - x_j) * x_j,
 *
 * K(y) = exp(-||y||^2 / sigma^2) (Gaussian, kernel 0) or exp(-||y|| / sigma)
 * (Laplacian RBF, kernel 1), the two kernels Sec. 4 names.
 *
 * The squared distance is summed in coordinate order from the differences
 * (x_ik - x_jk), so w_ij and w_ji are the same bits.  Each output uses
 * Neumaier's compensated summation over j in index order.  Rows are split
 * over OpenMP threads (static schedule); every row is independent, so the
 * result does not depend on the thread count.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static inline void neumaier_add(double *s, double *c, double v) {
    double t = *s + v;
    if (fabs(*s) >= fabs(v))
        *c += (*s - t) + v;
    else
        *c += (v - t) + *s;
    *s = t;
}

/*
 * points: n x d, row-major.  X: n x b column-major with leading dim ldx.
 * rows:   optional list of nrows row indices (NULL means rows 0..nrows-1).
 * Y:      nrows x b column-major with leading dim ldy.
 * Returns 0, or -1 for a bad argument.
 */
int oracle_kernel_rows_k(int64_t n, int d, const double *points, double sigma, int kernel,
                         int64_t nrows, const int64_t *rows, int b,
                         const double *X, int64_t ldx, double *Y, int64_t ldy) {
    if (n < 0 || d < 1 || sigma <= 0.0 || b < 1 || nrows < 0) return -1;
    if (kernel != 0 && kernel != 1) return -1;
    const double inv_s2 = 1.0 / (sigma * sigma);
    int bad = 0;
#pragma omp parallel
    {
        double *s = (double *)malloc(sizeof(double) * 2 * (size_t)b);
        double *c = s + b;
#pragma omp for schedule(static)
        for (int64_t r = 0; r < nrows; ++r) {
            int64_t i = rows ? rows[r] : r;
            if (i < 0 || i >= n) { bad = 1; continue; }
            for (int v = 0; v < b; ++v) { s[v] = 0.0; c[v] = 0.0; }
            const double *xi = points + i * d;
            for (int64_t j = 0; j < n; ++j) {
                if (j == i) continue;
                const double *xj = points + j * d;
                double r2 = 0.0;
                for (int k = 0; k < d; ++k) {
                    double dk = xi[k] - xj[k];
                    r2 += dk * dk;
                }
                double w = kernel == 0 ? exp(-r2 * inv_s2) : exp(-sqrt(r2) / sigma);
                for (int v = 0; v < b; ++v) neumaier_add(&s[v], &c[v], w * X[j + v * ldx]);
            }
            for (int v = 0; v < b; ++v) Y[r + v * ldy] = s[v] + c[v];
        }
        free(s);
    }
    return bad ? -1 : 0;
}

/* The Gaussian kernel (kernel 0). */
int oracle_kernel_rows(int64_t n, int d, const double *points, double sigma,
                       int64_t nrows, const int64_t *rows, int b,
                       const double *X, int64_t ldx, double *Y, int64_t ldy) {
    return oracle_kernel_rows_k(n, d, points, sigma, 0, nrows, rows, b, X, ldx, Y, ldy);
}
