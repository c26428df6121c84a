/*
 * Dense FP64 oracle for the GP log-likelihood.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The GPU product
 * path shares no code with it.
 *
 * It computes, by the plain definitions and nothing cleverer:
 *   C = sigma^2 I + K,  K_ij = k(x_i, x_j)           (§1: covariance of the form
 *                                                   sigma^2 I + K; Eq. (1))
 *   C = G G^T (Cholesky; C is symmetric positive definite, §1)
 *   log det C = 2 * sum_i log G_ii                 (pairwise summation)
 *   alpha = C^{-1} y = G^{-T} (G^{-1} y),  quad = y^T alpha
 *   loglik = -quad/2 - logdet/2 - (n/2) log(2 pi)  (Eq. (1) with the normal
 *                                                   density's constant, mean 0 as in §2.1)
 *
 * Kernels (Table 1 and §5; the length-scale/amplitude form is the usual one):
 *   0  squared exponential  a^2 exp(-r^2 / (2 l^2))
 *   1  Matern nu=3/2        a^2 (1 + sqrt(3) r / l) exp(-sqrt(3) r / l)
 *   2  exponential (O-U)    a^2 exp(-r / l)
 *   3  constant             a^2                       (rank one)
 *   4  inverse multiquadric a^2 / sqrt(1 + r^2 / l^2) (§5's inverse
 *                                                   multiquadric with a length scale)
 * with r the Euclidean distance between points.  Points are stored
 * point-major: x[i*dim + d].
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

double oracle_kernel(int kind, const double *xi, const double *xj, int dim,
                     double a, double ell)
{
    double r2 = 0.0;
    for (int d = 0; d < dim; ++d) {
        double t = xi[d] - xj[d];
        r2 += t * t;
    }
    double a2 = a * a;
    switch (kind) {
    case 0:
        return a2 * exp(-r2 / (2.0 * ell * ell));
    case 1: {
        double s = sqrt(3.0) * sqrt(r2) / ell;
        return a2 * (1.0 + s) * exp(-s);
    }
    case 2:
        return a2 * exp(-sqrt(r2) / ell);
    case 3:
        return a2;
    case 4: /* inverse multiquadric (§5), with a length scale */
        return a2 / sqrt(1.0 + r2 / (ell * ell));
    default:
        return NAN;
    }
}

/* Cross matrix K(xa, xb) (no noise term), row-major na x nb:
 * out[i * nb + j] = k(xa_i, xb_j), point-major inputs.  The prediction of
 * §2.1 needs it with xa the new inputs and xb the data. */
void oracle_cross_matrix(const double *xa, int64_t na, const double *xb, int64_t nb, int dim,
                         int kind, double a, double ell, double *out)
{
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < na; ++i)
        for (int64_t j = 0; j < nb; ++j)
            out[i * nb + j] = oracle_kernel(kind, xa + i * dim, xb + j * dim, dim, a, ell);
}

/* Full symmetric matrix C = sigma2*I + K, row-major n x n. */
void oracle_dense_matrix(const double *x, int64_t n, int dim, int kind, double a,
                         double ell, double sigma2, double *C)
{
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i) {
        for (int64_t j = 0; j < n; ++j) {
            double v = oracle_kernel(kind, x + i * dim, x + j * dim, dim, a, ell);
            if (i == j)
                v += sigma2;
            C[i * n + j] = v;
        }
    }
}

static double dot(const double *u, const double *v, int64_t m)
{
    double s = 0.0;
    for (int64_t k = 0; k < m; ++k)
        s += u[k] * v[k];
    return s;
}

/*
 * In-place Cholesky C = G G^T (column-by-column, Crout order).  The lower
 * triangle of C is overwritten with G; the strict upper triangle is zeroed.
 * Returns 0 on success, or 1 + j when the pivot of column j is not positive.
 */
int oracle_cholesky(double *C, int64_t n)
{
    for (int64_t j = 0; j < n; ++j) {
        double *rj = C + j * n;
        double d = rj[j] - dot(rj, rj, j);
        if (!(d > 0.0))
            return (int)(j + 1);
        double gjj = sqrt(d);
        rj[j] = gjj;
#pragma omp parallel for schedule(static)
        for (int64_t i = j + 1; i < n; ++i) {
            double *ri = C + i * n;
            ri[j] = (ri[j] - dot(ri, rj, j)) / gjj;
        }
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t j = i + 1; j < n; ++j)
            C[i * n + j] = 0.0;
    return 0;
}

/* Pairwise sum of v[0..m). */
static double pairwise_sum(const double *v, int64_t m)
{
    if (m <= 8) {
        double s = 0.0;
        for (int64_t k = 0; k < m; ++k)
            s += v[k];
        return s;
    }
    int64_t h = m / 2;
    return pairwise_sum(v, h) + pairwise_sum(v + h, m - h);
}

double oracle_logdet_chol(const double *G, int64_t n)
{
    double *lg = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    for (int64_t i = 0; i < n; ++i)
        lg[i] = log(G[i * n + i]);
    double s = 2.0 * pairwise_sum(lg, n);
    free(lg);
    return s;
}

/* x = C^{-1} b with C = G G^T: forward then backward substitution. */
void oracle_chol_solve(const double *G, int64_t n, const double *b, double *x)
{
    for (int64_t i = 0; i < n; ++i)
        x[i] = (b[i] - dot(G + i * n, x, i)) / G[i * n + i];
    for (int64_t i = n - 1; i >= 0; --i) {
        double s = x[i];
        for (int64_t k = i + 1; k < n; ++k)
            s -= G[k * n + i] * x[k];
        x[i] = s / G[i * n + i];
    }
}

/*
 * Whole GP evaluation.  Outputs are written only on success.
 * Returns 0 on success, -1 on allocation failure, or 1 + j when C is not
 * positive definite (Cholesky pivot j failed).
 */
int oracle_gp(const double *x, int64_t n, int dim, int kind, double a, double ell,
              double sigma2, const double *y, double *logdet, double *quad,
              double *loglik, double *alpha)
{
    double *C = (double *)malloc(sizeof(double) * (size_t)n * (size_t)n);
    double *al = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!C || !al) {
        free(C);
        free(al);
        return -1;
    }
    oracle_dense_matrix(x, n, dim, kind, a, ell, sigma2, C);
    int st = oracle_cholesky(C, n);
    if (st != 0) {
        free(C);
        free(al);
        return st;
    }
    double ld = oracle_logdet_chol(C, n);
    oracle_chol_solve(C, n, y, al);
    double q = dot(y, al, n);
    if (logdet)
        *logdet = ld;
    if (quad)
        *quad = q;
    if (loglik)
        *loglik = -0.5 * q - 0.5 * ld - 0.5 * (double)n * log(2.0 * M_PI);
    if (alpha)
        memcpy(alpha, al, sizeof(double) * (size_t)n);
    free(C);
    free(al);
    return 0;
}

/*
 * out[k] = (C v)[rows[k]] with C evaluated entry by entry (never stored):
 * the exact operator used for residuals ||y - C x|| at sizes where C
 * cannot be formed.
 */
void oracle_matvec_rows(const double *x, int64_t n, int dim, int kind, double a,
                        double ell, double sigma2, const double *v,
                        const int64_t *rows, int64_t nrows, double *out)
{
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t k = 0; k < nrows; ++k) {
        int64_t i = rows[k];
        double s = 0.0;
        for (int64_t j = 0; j < n; ++j)
            s += oracle_kernel(kind, x + i * dim, x + j * dim, dim, a, ell) * v[j];
        out[k] = s + sigma2 * v[i];
    }
}
