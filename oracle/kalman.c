/*
 * Exact O(n) reference for 1-D Matern-3/2 GPs via the state-space view.
 *
 * TEST INFRASTRUCTURE ONLY (same rules as dense_oracle.c).
 *
 * §2.4 of the paper notes that stationary kernels with rational spectra
 * admit a linear state-space (Kalman filter) form with O(n) inference.  For
 * the Matern nu=3/2 kernel k(r) = a^2 (1 + lam r) exp(-lam r), lam = sqrt(3)/l,
 * the latent state s = (f, f') obeys
 *     s(t+dt) = A(dt) s(t) + q,   q ~ N(0, Q(dt)),
 *     A(dt) = exp(-lam dt) [[1 + lam dt, dt], [-lam^2 dt, 1 - lam dt]],
 *     P_inf = diag(a^2, lam^2 a^2),   Q = P_inf - A P_inf A^T,
 * and y_i = f(t_i) + e_i with e_i ~ N(0, s_i), s_i = sigma^2 (+ a per-point
 * variance sigma_i^2 when one is given: §5 writes the diagonal of C as
 * sigma_i^2).  The filter's innovations v_i and their variances S_i give the
 * exact Gaussian quantities
 *     log det C = sum_i log S_i,     y^T C^{-1} y = sum_i v_i^2 / S_i,
 * and the Rauch-Tung-Striebel smoothed mean m_s gives
 *     C^{-1} y = D^{-1} (y - m_s)   (since Cov(e, y) = D = diag(s_i)).
 * Times must be sorted ascending.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

typedef struct {
    double a00, a01, a10, a11;
} m22;

static m22 trans(double lam, double dt)
{
    double e = exp(-lam * dt);
    m22 A = {e * (1.0 + lam * dt), e * dt, -e * lam * lam * dt, e * (1.0 - lam * dt)};
    return A;
}

/* P' = A P A^T (P symmetric, stored p00 p01 p11) */
static void sandwich(const m22 *A, const double *P, double *out)
{
    double t00 = A->a00 * P[0] + A->a01 * P[1];
    double t01 = A->a00 * P[1] + A->a01 * P[2];
    double t10 = A->a10 * P[0] + A->a11 * P[1];
    double t11 = A->a10 * P[1] + A->a11 * P[2];
    out[0] = t00 * A->a00 + t01 * A->a01;
    out[1] = t00 * A->a10 + t01 * A->a11;
    out[2] = t10 * A->a10 + t11 * A->a11;
}

/*
 * Returns 0 on success, 1 on bad arguments (unsorted times, a noise variance
 * <= 0 when alpha is requested, non-positive innovation variance), -1 on
 * allocation failure.  alpha (C^{-1} y) may be NULL; noise (per-point
 * variances added to sigma2) may be NULL.
 */
int oracle_kalman_matern32_noise(const double *t, int64_t n, double a, double ell,
                                 double sigma2, const double *noise, const double *y,
                                 double *logdet, double *quad, double *alpha)
{
    if (n < 1)
        return 1;
    for (int64_t i = 1; i < n; ++i)
        if (!(t[i] >= t[i - 1]))
            return 1;
    for (int64_t i = 0; i < n; ++i) {
        const double si = sigma2 + (noise ? noise[i] : 0.0);
        if (alpha && !(si > 0.0))
            return 1;
    }
    double lam = sqrt(3.0) / ell;
    double pinf[3] = {a * a, 0.0, lam * lam * a * a};
    /* filtered and predicted moments, kept for the smoother */
    double *mf = NULL, *Pf = NULL, *mp = NULL, *Pp = NULL;
    if (alpha) {
        mf = (double *)malloc(sizeof(double) * 2 * (size_t)n);
        mp = (double *)malloc(sizeof(double) * 2 * (size_t)n);
        Pf = (double *)malloc(sizeof(double) * 3 * (size_t)n);
        Pp = (double *)malloc(sizeof(double) * 3 * (size_t)n);
        if (!mf || !mp || !Pf || !Pp) {
            free(mf); free(mp); free(Pf); free(Pp);
            return -1;
        }
    }
    double m[2] = {0.0, 0.0};
    double P[3] = {pinf[0], pinf[1], pinf[2]};
    double ld = 0.0, q = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        double mpr[2], Ppr[3];
        if (i == 0) {
            mpr[0] = 0.0; mpr[1] = 0.0;
            Ppr[0] = pinf[0]; Ppr[1] = pinf[1]; Ppr[2] = pinf[2];
        } else {
            m22 A = trans(lam, t[i] - t[i - 1]);
            mpr[0] = A.a00 * m[0] + A.a01 * m[1];
            mpr[1] = A.a10 * m[0] + A.a11 * m[1];
            double APA[3], Api[3];
            sandwich(&A, P, APA);
            sandwich(&A, pinf, Api);
            Ppr[0] = APA[0] + (pinf[0] - Api[0]);
            Ppr[1] = APA[1] + (pinf[1] - Api[1]);
            Ppr[2] = APA[2] + (pinf[2] - Api[2]);
        }
        double S = Ppr[0] + sigma2 + (noise ? noise[i] : 0.0);
        if (!(S > 0.0)) {
            if (alpha) { free(mf); free(mp); free(Pf); free(Pp); }
            return 1;
        }
        double v = y[i] - mpr[0];
        double k0 = Ppr[0] / S, k1 = Ppr[1] / S;
        m[0] = mpr[0] + k0 * v;
        m[1] = mpr[1] + k1 * v;
        P[0] = Ppr[0] - k0 * S * k0;
        P[1] = Ppr[1] - k0 * S * k1;
        P[2] = Ppr[2] - k1 * S * k1;
        ld += log(S);
        q += v * v / S;
        if (alpha) {
            mp[2 * i] = mpr[0]; mp[2 * i + 1] = mpr[1];
            Pp[3 * i] = Ppr[0]; Pp[3 * i + 1] = Ppr[1]; Pp[3 * i + 2] = Ppr[2];
            mf[2 * i] = m[0]; mf[2 * i + 1] = m[1];
            Pf[3 * i] = P[0]; Pf[3 * i + 1] = P[1]; Pf[3 * i + 2] = P[2];
        }
    }
    if (logdet)
        *logdet = ld;
    if (quad)
        *quad = q;
    if (alpha) {
        /* RTS backward pass for the smoothed mean of f */
        double ms0 = mf[2 * (n - 1)], ms1 = mf[2 * (n - 1) + 1];
        alpha[n - 1] = (y[n - 1] - ms0) / (sigma2 + (noise ? noise[n - 1] : 0.0));
        for (int64_t i = n - 2; i >= 0; --i) {
            m22 A = trans(lam, t[i + 1] - t[i]);
            const double *Pi = Pf + 3 * i;
            const double *Pn = Pp + 3 * (i + 1);
            /* G = P_i A^T Pn^{-1} */
            double c00 = Pi[0] * A.a00 + Pi[1] * A.a01;
            double c01 = Pi[0] * A.a10 + Pi[1] * A.a11;
            double c10 = Pi[1] * A.a00 + Pi[2] * A.a01;
            double c11 = Pi[1] * A.a10 + Pi[2] * A.a11;
            double det = Pn[0] * Pn[2] - Pn[1] * Pn[1];
            double i00 = Pn[2] / det, i01 = -Pn[1] / det, i11 = Pn[0] / det;
            double g00 = c00 * i00 + c01 * i01, g01 = c00 * i01 + c01 * i11;
            double g10 = c10 * i00 + c11 * i01, g11 = c10 * i01 + c11 * i11;
            double d0 = ms0 - mp[2 * (i + 1)], d1 = ms1 - mp[2 * (i + 1) + 1];
            double n0 = mf[2 * i] + g00 * d0 + g01 * d1;
            double n1 = mf[2 * i + 1] + g10 * d0 + g11 * d1;
            ms0 = n0;
            ms1 = n1;
            alpha[i] = (y[i] - ms0) / (sigma2 + (noise ? noise[i] : 0.0));
        }
        free(mf); free(mp); free(Pf); free(Pp);
    }
    return 0;
}

int oracle_kalman_matern32(const double *t, int64_t n, double a, double ell,
                           double sigma2, const double *y, double *logdet,
                           double *quad, double *alpha)
{
    return oracle_kalman_matern32_noise(t, n, a, ell, sigma2, NULL, y, logdet, quad, alpha);
}
