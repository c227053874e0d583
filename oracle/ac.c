/*
 * ORACLE -- test infrastructure only.  Only tests/, the smoke entry and the
 * benchmark's CPU-baseline leg may load this code; the GPU library never does.
 *
 * Multiclass Allen--Cahn scheme in the truncated eigenbasis (Algorithm 2,
 * steps 2-4; scheme of Sec. 5 with the multilayer operator of Sec. 6; the
 * eigenbasis iteration of Appendix B), FP64, in one fixed operation order so
 * that a second implementation following the same order gives the same bits.
 * Built with -ffp-contract=off: every product is rounded before it is added.
 *
 * Canonical order (both implementations follow it):
 *   denominator  den_r = (1 + c*dt) + (eps*dt)*lambda_r, Z_ri = phi_ir / den_r
 *   potential    a_q = sum_c |u_ic - delta_qc|           (c ascending)
 *                s_p = 0.25*(a_p*a_p)
 *                term_q = (0.5*a_q) * prod_{p != q} s_p  (p ascending)
 *                T_ij = sum_q (q == j ? -term_q : +term_q)  (q ascending)
 *   right side   R = ((1+c*dt)*U - (dt/(2*eps))*T) - (dt*omega_i)*(U - F)
 *   V = Z R      rows in chunks of 256, each chunk summed in row order, then
 *                a pairwise tree over chunks: level by level, neighbours
 *                (2j, 2j+1) added, an odd last element carried up unchanged
 *   U~ = Phi V   sum over r ascending
 *   projection   Chen & Ye (2011) onto the Gibbs simplex, sums from the top
 *   change       max_i ||u_i^new - u_i^old||^2 / max_i ||u_i^new||^2
 *   prediction   row argmax, the lowest class id wins ties (Sec. 6)
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define AC_CHUNK 256

typedef struct {
    double eps, omega0, c, dt, tol;
    int max_iter;
} oracle_ac_params;

/* Projection of y (length m) onto {x >= 0, sum x = 1}, Chen & Ye 2011:
 * sort ascending; for i = m-1 .. 1 (1-based) t_i = (sum_{j>i} y_(j) - 1)/(m-i);
 * the first t_i >= y_(i) is t^; otherwise t^ = (sum_j y_j - 1)/m;
 * x = max(y - t^, 0). */
void oracle_simplex_project(int m, const double *y, double *x) {
    double srt[64];
    for (int i = 0; i < m; ++i) {
        double v = y[i];
        int j = i - 1;
        while (j >= 0 && srt[j] > v) { srt[j + 1] = srt[j]; --j; }
        srt[j + 1] = v;
    }
    double s = 0.0, that = 0.0;
    int found = 0;
    for (int i = m - 1; i >= 1; --i) {          /* 1-based i; srt[i] = y_(i+1) */
        s = s + srt[i];
        double t = (s - 1.0) / (double)(m - i);
        if (t >= srt[i - 1]) { that = t; found = 1; break; }
    }
    if (!found) {
        s = s + srt[0];
        that = (s - 1.0) / (double)m;
    }
    for (int i = 0; i < m; ++i) {
        double dlt = y[i] - that;
        x[i] = dlt > 0.0 ? dlt : 0.0;
    }
}

/* Derivative of the multi-well potential, entries T_ij (Sec. 5). */
void oracle_potential_grad(int m, const double *u, double *T) {
    double a[64], s[64], term[64];
    for (int q = 0; q < m; ++q) {
        double acc = 0.0;
        for (int c = 0; c < m; ++c) acc = acc + fabs(u[c] - (c == q ? 1.0 : 0.0));
        a[q] = acc;
        s[q] = 0.25 * (a[q] * a[q]);
    }
    for (int q = 0; q < m; ++q) {
        double prod = 1.0;
        for (int p = 0; p < m; ++p)
            if (p != q) prod = prod * s[p];
        term[q] = (0.5 * a[q]) * prod;
    }
    for (int j = 0; j < m; ++j) {
        double t = 0.0;
        for (int q = 0; q < m; ++q) t = (q == j) ? t - term[q] : t + term[q];
        T[j] = t;
    }
}

/* Pairwise tree over `cnt` partial results of length len stored back to back;
 * the result lands in p[0..len). */
static void tree_sum(double *p, int64_t cnt, int len) {
    while (cnt > 1) {
        int64_t half = cnt / 2;
        for (int64_t j = 0; j < half; ++j)
            for (int e = 0; e < len; ++e)
                p[j * len + e] = p[(2 * j) * len + e] + p[(2 * j + 1) * len + e];
        if (cnt & 1)
            for (int e = 0; e < len; ++e) p[half * len + e] = p[(cnt - 1) * len + e];
        cnt = half + (cnt & 1);
    }
}

/*
 * evals: k eigenvalues lambda_r of the Laplacian (ascending, not required).
 * evecs: n x k column-major, leading dim ldv.
 * labels: n entries, -1 = unlabelled, 0..m-1 = class.
 * U: n x m row-major output scores; pred: n labels; iters: iterations run;
 * min_margin: smallest top-two score gap over all rows (diagnostic).
 * Returns 0, or -1 for a bad argument.
 */
int oracle_allen_cahn(int64_t n, int k, int m, const double *evals, const double *evecs,
                      int64_t ldv, const int32_t *labels, const oracle_ac_params *prm,
                      double *U, int32_t *pred, int *iters, double *min_margin) {
    if (n < 1 || k < 1 || m < 2 || m > 64 || ldv < n) return -1;
    const double eps = prm->eps, dt = prm->dt, c = prm->c, om0 = prm->omega0;
    double onepcdt = c * dt;
    onepcdt = 1.0 + onepcdt;
    const double epsdt = eps * dt;
    const double coefT = dt / (2.0 * eps);

    double *Z = (double *)malloc(sizeof(double) * (size_t)k * (size_t)n);
    for (int r = 0; r < k; ++r) {
        double e = epsdt * evals[r];
        double den = onepcdt + e;
        for (int64_t i = 0; i < n; ++i) Z[(int64_t)r * n + i] = evecs[i + (int64_t)r * ldv] / den;
    }
    double *F = (double *)calloc((size_t)n * m, sizeof(double));
    double *om = (double *)malloc(sizeof(double) * (size_t)n);
    const double inv_m = 1.0 / (double)m;
    for (int64_t i = 0; i < n; ++i) {
        int l = labels[i];
        if (l >= m) { free(Z); free(F); free(om); return -1; }
        om[i] = (l >= 0) ? om0 : 0.0;
        for (int j = 0; j < m; ++j) {
            F[i * m + j] = (l >= 0 && j == l) ? 1.0 : 0.0;
            U[i * m + j] = (l >= 0) ? F[i * m + j] : inv_m;
        }
    }
    double *R = (double *)malloc(sizeof(double) * (size_t)n * m);
    int64_t nch = (n + AC_CHUNK - 1) / AC_CHUNK;
    double *part = (double *)malloc(sizeof(double) * (size_t)nch * k * m);
    double *Ut = (double *)malloc(sizeof(double) * (size_t)m);
    double T[64];
    int l = 0;
    double rc = 0.0;
    do {
        /* (a) T(U^l) and the right-hand side */
        for (int64_t i = 0; i < n; ++i) {
            oracle_potential_grad(m, U + i * m, T);
            double w = dt * om[i];
            for (int j = 0; j < m; ++j) {
                double u = U[i * m + j];
                double r1 = onepcdt * u;
                double r2 = coefT * T[j];
                double r3 = r1 - r2;
                double r4 = u - F[i * m + j];
                double r5 = w * r4;
                R[i * m + j] = r3 - r5;
            }
        }
        /* (b) V = Z R, chunked then pairwise */
        for (int64_t ch = 0; ch < nch; ++ch) {
            int64_t i0 = ch * AC_CHUNK, i1 = i0 + AC_CHUNK < n ? i0 + AC_CHUNK : n;
            for (int r = 0; r < k; ++r)
                for (int j = 0; j < m; ++j) {
                    double acc = 0.0;
                    for (int64_t i = i0; i < i1; ++i) {
                        double pr = Z[(int64_t)r * n + i] * R[i * m + j];
                        acc = acc + pr;
                    }
                    part[(ch * k + r) * m + j] = acc;
                }
        }
        tree_sum(part, nch, k * m);
        /* (c) U~ = Phi V, projection, relative change */
        double num = 0.0, den = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            for (int j = 0; j < m; ++j) {
                double acc = 0.0;
                for (int r = 0; r < k; ++r) {
                    double pr = evecs[i + (int64_t)r * ldv] * part[r * m + j];
                    acc = acc + pr;
                }
                Ut[j] = acc;
            }
            double un[64];
            oracle_simplex_project(m, Ut, un);
            double dn = 0.0, nn = 0.0;
            for (int j = 0; j < m; ++j) {
                double dl = un[j] - U[i * m + j];
                double p1 = dl * dl;
                dn = dn + p1;
                double p2 = un[j] * un[j];
                nn = nn + p2;
                U[i * m + j] = un[j];
            }
            if (dn > num) num = dn;
            if (nn > den) den = nn;
        }
        rc = num / den;
        l = l + 1;
    } while (rc > prm->tol && l < prm->max_iter);

    double mm = INFINITY;
    for (int64_t i = 0; i < n; ++i) {
        int best = 0;
        for (int j = 1; j < m; ++j)
            if (U[i * m + j] > U[i * m + best]) best = j;
        pred[i] = best;
        double second = -INFINITY;
        for (int j = 0; j < m; ++j)
            if (j != best && U[i * m + j] > second) second = U[i * m + j];
        double g = U[i * m + best] - second;
        if (g < mm) mm = g;
    }
    if (iters) *iters = l;
    if (min_margin) *min_margin = mm;
    free(Z); free(F); free(om); free(R); free(part); free(Ut);
    return 0;
}
