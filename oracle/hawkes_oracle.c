/*
 * Plain FP64 CPU oracle for the spatiotemporal Hawkes log-likelihood with
 * per-event rates (Holbrook, Ji & Suchard, "From viral evolution to spatial
 * contagion: a biologically modulated Hawkes model", arXiv 2103.03348).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the correctness reference that the
 * GPU library is checked against.  It is compiled into liboracle.so, which only
 * the test suite, the smoke check and the CPU-baseline leg of the benchmark may
 * load.  It shares no source with the HIP library.
 *
 * What is computed (D = 2 spatial dimensions, events n = 1..N, window [T0, T1],
 * T1 = max_n t_n):
 *
 *   b_ij = exp(-|x_i-x_j|^2 / (2 tau_x^2) - (t_i-t_j)^2 / (2 tau_t^2))   all j != i
 *   E_ij = exp(-omega (t_i-t_j) - |x_i-x_j|^2 / (2 h^2))                 t_j < t_i
 *   c_b  = mu0 / ((2 pi)^{3/2} tau_x^2 tau_t),   c_e = theta0 omega / (2 pi h^2)
 *   lambda_i = c_b sum_{j != i} b_ij + c_e sum_{t_j < t_i} theta_j E_ij
 *
 * Sec. 2.1 gives the intensity: a background kernel density over all other
 * events (self-excluded, no causal indicator) plus a causal, exponential-in-time,
 * Gaussian-in-space excitation scaled by theta0 * theta_n.  The paper's
 * background is Gaussian in space only; the temporal factor
 * tau_t^{-1} phi((t_i - t_j)/tau_t) is this library's extension (reading C1).
 * The self-exclusion indicator is read as j != i (reading C3).  Excitation is
 * strict in time: tied events do not excite each other (reading C4).
 *
 *   Lambda = mu0 sum_n [Phi((T1-t_n)/tau_t) - Phi((T0-t_n)/tau_t)]
 *          + theta0 sum_n theta_n (1 - exp(-omega (T1 - t_n)))
 *
 * The excitation part is Appendix A's claim; the background part is the exact
 * integral of the stated background over R^2 x [T0, T1] (reading C2: the paper's
 * mu0 * t_N is not the integral of its own spatial kernel density).
 *
 *   loglik = sum_i log lambda_i - Lambda                       (Eq. 1)
 *   ell_n  = log lambda_n - Lambda_n   (per-event split of Eq. 1)
 *   d loglik / d theta_j    = sum_{t_i > t_j} c_e E_ij / lambda_i
 *                             - theta0 (1 - exp(-omega (T1 - t_j)))   (Eq. 4)
 *   -d2 loglik / d theta_j^2 = sum_{t_i > t_j} (c_e E_ij / lambda_i)^2 (Eq. 5,
 *                             exact because lambda_i and Lambda are linear in theta_j)
 *
 * Hyperparameter derivatives (mu0, tau_x, tau_t, theta0, omega, h) are not in
 * the paper (its hyperparameters are sampled by Metropolis-Hastings, Sec. 2.3.2);
 * they are obtained here by differentiating the definitions above, each line
 * below stating the derivative it takes.
 *
 * Implementation rules: i-outer / j-inner double loops over the events in the
 * order given (no sorting, tiling or reordering), libm exp/log/erfc, FP64
 * throughout, OpenMP over the outer index, Neumaier summation for the final
 * sums over events.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORACLE_PI 3.14159265358979323846

/* Standard normal density and cdf (Phi via erfc for accuracy in both tails). */
static double std_phi(double u) { return exp(-0.5 * u * u) / sqrt(2.0 * ORACLE_PI); }
static double std_Phi(double u) { return 0.5 * erfc(-u / sqrt(2.0)); }

/* Neumaier compensated sum of v[0..n-1]; an infinite or NaN term makes the
   plain sum the answer (the compensation would turn -inf into NaN). */
static double neumaier(const double *v, int64_t n) {
    double s = 0.0, c = 0.0, plain = 0.0;
    for (int64_t k = 0; k < n; ++k) {
        double t = s + v[k];
        plain += v[k];
        if (fabs(s) >= fabs(v[k])) c += (s - t) + v[k];
        else c += (v[k] - t) + s;
        s = t;
    }
    if (!isfinite(plain)) return plain;
    return s + c;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Per-row pair sums for rows rows[0..nrows-1] (or all rows when rows == NULL,
 * nrows == n).  acc is [nrows][10]:
 *   0 B0  = sum_{j!=i} b_ij          1 B1  = sum b r^2      2 B2  = sum b dt^2
 *   3 B11 = sum b r^4                4 B22 = sum b dt^4
 *   5 X0  = sum_{t_j<t_i} theta_j E_ij
 *   6 X1  = sum theta E dt           7 X2  = sum theta E r^2
 *   8 X11 = sum theta E dt^2         9 X22 = sum theta E r^4
 */
int oracle_row_sums(int64_t n, const double *t, const double *x, const double *y,
                    const double *theta, const double *hyper,
                    int64_t nrows, const int64_t *rows, double *acc, int nthreads) {
    const double tau_x = hyper[1], tau_t = hyper[2], omega = hyper[4], h = hyper[5];
    if (nthreads <= 0) nthreads = oracle_max_threads();
    int64_t k;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (k = 0; k < nrows; ++k) {
        int64_t i = rows ? rows[k] : k;
        double s[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dt = t[i] - t[j];
            double r2 = dx * dx + dy * dy;
            double b = exp(-r2 / (2.0 * tau_x * tau_x) - dt * dt / (2.0 * tau_t * tau_t));
            s[0] += b;
            s[1] += b * r2;
            s[2] += b * dt * dt;
            s[3] += b * r2 * r2;
            s[4] += b * dt * dt * dt * dt;
            if (t[j] < t[i]) {
                double e = theta[j] * exp(-omega * dt - r2 / (2.0 * h * h));
                s[5] += e;
                s[6] += e * dt;
                s[7] += e * r2;
                s[8] += e * dt * dt;
                s[9] += e * r2 * r2;
            }
        }
        memcpy(acc + 10 * k, s, sizeof(s));
    }
    return 0;
}

/*
 * Column sums of Eq. 4 and Eq. 5 for columns cols[0..ncols-1] (all when NULL),
 * given lambda for every event: G_j = sum_{t_i>t_j} c_e E_ij / lambda_i and
 * H_j = sum_{t_i>t_j} (c_e E_ij / lambda_i)^2.
 */
int oracle_col_sums(int64_t n, const double *t, const double *x, const double *y,
                    const double *hyper, const double *lam,
                    int64_t ncols, const int64_t *cols, double *G, double *H, int nthreads) {
    const double theta0 = hyper[3], omega = hyper[4], h = hyper[5];
    const double c_e = theta0 * omega / (2.0 * ORACLE_PI * h * h);
    if (nthreads <= 0) nthreads = oracle_max_threads();
    int64_t k;
#pragma omp parallel for schedule(dynamic, 16) num_threads(nthreads)
    for (k = 0; k < ncols; ++k) {
        int64_t j = cols ? cols[k] : k;
        double g = 0.0, hh = 0.0;
        for (int64_t i = 0; i < n; ++i) {
            if (!(t[j] < t[i])) continue;
            double dx = x[i] - x[j], dy = y[i] - y[j], dt = t[i] - t[j];
            double r2 = dx * dx + dy * dy;
            double a = c_e * exp(-omega * dt - r2 / (2.0 * h * h)) / lam[i];
            g += a;
            hh += a * a;
        }
        G[k] = g;
        H[k] = hh;
    }
    return 0;
}

/*
 * Full evaluation.  Every output pointer may be NULL.
 *   lam[n], ell_n[n], Lam_n[n], grad_theta[n], negH_theta[n],
 *   grad_hyper[6], negH_hyper[6], loglik[1]
 * hyper = (mu0, tau_x, tau_t, theta0, omega, h).  T0 is the window start.
 * Returns 0, or 1 if the arguments are invalid.
 */
int oracle_eval(int64_t n, const double *t, const double *x, const double *y,
                const double *theta, const double *hyper, double T0,
                double *lam, double *ell_n, double *Lam_n,
                double *grad_theta, double *negH_theta,
                double *grad_hyper, double *negH_hyper, double *loglik, int nthreads) {
    if (n < 1) return 1;
    const double mu0 = hyper[0], tau_x = hyper[1], tau_t = hyper[2];
    const double theta0 = hyper[3], omega = hyper[4], h = hyper[5];
    if (!(tau_x > 0 && tau_t > 0 && omega > 0 && h > 0 && mu0 >= 0 && theta0 >= 0)) return 1;
    double T1 = t[0];
    for (int64_t i = 1; i < n; ++i) if (t[i] > T1) T1 = t[i];

    /* unit-weight normalisers, so that derivatives in mu0 and theta0 stay defined at 0 */
    const double cb1 = 1.0 / (pow(2.0 * ORACLE_PI, 1.5) * tau_x * tau_x * tau_t);
    const double ce1 = omega / (2.0 * ORACLE_PI * h * h);
    const double c_b = mu0 * cb1;
    const double c_e = theta0 * ce1;

    double *acc = (double *)malloc(sizeof(double) * 10 * (size_t)n);
    double *lam_ = (double *)malloc(sizeof(double) * (size_t)n);
    double *tmp = (double *)malloc(sizeof(double) * 13 * (size_t)n);
    if (!acc || !lam_ || !tmp) { free(acc); free(lam_); free(tmp); return 2; }
    oracle_row_sums(n, t, x, y, theta, hyper, n, NULL, acc, nthreads);

    /* per-event terms; tmp columns: 0 log lambda, 1..6 lambda'/lambda, 7..12 lambda''/lambda */
    for (int64_t i = 0; i < n; ++i) {
        const double *s = acc + 10 * i;
        double l = c_b * s[0] + c_e * s[5];
        lam_[i] = l;
        double d1[6], d2[6];
        /* d/d mu0: c_b is linear in mu0 */
        d1[0] = cb1 * s[0];                                               d2[0] = 0.0;
        /* d/d tau_x: c_b ~ tau_x^-2, b ~ exp(-r^2/(2 tau_x^2)) */
        d1[1] = c_b * (-2.0 * s[0] / tau_x + s[1] / pow(tau_x, 3));
        d2[1] = c_b * (6.0 * s[0] / pow(tau_x, 2) - 7.0 * s[1] / pow(tau_x, 4) + s[3] / pow(tau_x, 6));
        /* d/d tau_t: c_b ~ tau_t^-1, b ~ exp(-dt^2/(2 tau_t^2)) */
        d1[2] = c_b * (-s[0] / tau_t + s[2] / pow(tau_t, 3));
        d2[2] = c_b * (2.0 * s[0] / pow(tau_t, 2) - 5.0 * s[2] / pow(tau_t, 4) + s[4] / pow(tau_t, 6));
        /* d/d theta0: c_e is linear in theta0 */
        d1[3] = ce1 * s[5];                                               d2[3] = 0.0;
        /* d/d omega: c_e ~ omega, E ~ exp(-omega dt) */
        d1[4] = c_e * (s[5] / omega - s[6]);
        d2[4] = c_e * (s[8] - 2.0 * s[6] / omega);
        /* d/d h: c_e ~ h^-2, E ~ exp(-r^2/(2 h^2)) */
        d1[5] = c_e * (-2.0 * s[5] / h + s[7] / pow(h, 3));
        d2[5] = c_e * (6.0 * s[5] / pow(h, 2) - 7.0 * s[7] / pow(h, 4) + s[9] / pow(h, 6));
        tmp[13 * i + 0] = log(l);
        for (int p = 0; p < 6; ++p) {
            tmp[13 * i + 1 + p] = d1[p] / l;
            tmp[13 * i + 7 + p] = d2[p] / l;
        }
    }

    /* Integral term per event and its hyperparameter derivatives. */
    double *ig = (double *)malloc(sizeof(double) * 11 * (size_t)n);
    for (int64_t n_ = 0; n_ < n; ++n_) {
        double u1 = (T1 - t[n_]) / tau_t, u0 = (T0 - t[n_]) / tau_t;
        double s = T1 - t[n_];
        double es = exp(-omega * s);
        double C = std_Phi(u1) - std_Phi(u0);
        double *g = ig + 11 * n_;
        g[0] = mu0 * C + theta0 * theta[n_] * (1.0 - es);                 /* Lambda_n            */
        g[1] = C;                                                         /* dLambda/dmu0        */
        g[2] = mu0 * (-std_phi(u1) * u1 + std_phi(u0) * u0) / tau_t;      /* dLambda/dtau_t      */
        g[3] = theta[n_] * (1.0 - es);                                    /* dLambda/dtheta0     */
        g[4] = theta0 * theta[n_] * s * es;                               /* dLambda/domega      */
        g[5] = mu0 * (std_phi(u1) * (2.0 * u1 - u1 * u1 * u1)
                      - std_phi(u0) * (2.0 * u0 - u0 * u0 * u0)) / (tau_t * tau_t); /* d2/dtau_t2 */
        g[6] = -theta0 * theta[n_] * s * s * es;                          /* d2Lambda/domega2    */
        g[7] = theta0 * (1.0 - es);                                       /* dLambda/dtheta_n    */
    }

    double *col = (double *)malloc(sizeof(double) * (size_t)n);
    /* log-likelihood and the per-event split */
    for (int64_t i = 0; i < n; ++i) col[i] = tmp[13 * i];
    double sum_log = neumaier(col, n);
    for (int64_t i = 0; i < n; ++i) col[i] = ig[11 * i];
    double Lam = neumaier(col, n);
    if (loglik) loglik[0] = sum_log - Lam;
    if (lam) memcpy(lam, lam_, sizeof(double) * (size_t)n);
    if (ell_n) for (int64_t i = 0; i < n; ++i) ell_n[i] = tmp[13 * i] - ig[11 * i];
    if (Lam_n) for (int64_t i = 0; i < n; ++i) Lam_n[i] = ig[11 * i];

    if (grad_hyper || negH_hyper) {
        /* map hyper index -> integral-derivative slots (first, second) */
        const int d1slot[6] = {1, -1, 2, 3, 4, -1};
        const int d2slot[6] = {-1, -1, 5, -1, 6, -1};
        for (int p = 0; p < 6; ++p) {
            for (int64_t i = 0; i < n; ++i) col[i] = tmp[13 * i + 1 + p];
            double s1 = neumaier(col, n);
            for (int64_t i = 0; i < n; ++i) {
                double r = tmp[13 * i + 1 + p];
                col[i] = tmp[13 * i + 7 + p] - r * r;
            }
            double s2 = neumaier(col, n);
            double L1 = 0.0, L2 = 0.0;
            if (d1slot[p] >= 0) { for (int64_t i = 0; i < n; ++i) col[i] = ig[11 * i + d1slot[p]]; L1 = neumaier(col, n); }
            if (d2slot[p] >= 0) { for (int64_t i = 0; i < n; ++i) col[i] = ig[11 * i + d2slot[p]]; L2 = neumaier(col, n); }
            if (grad_hyper) grad_hyper[p] = s1 - L1;
            if (negH_hyper) negH_hyper[p] = -s2 + L2;
        }
    }

    if (grad_theta || negH_theta) {
        double *G = (double *)malloc(sizeof(double) * (size_t)n);
        double *H = (double *)malloc(sizeof(double) * (size_t)n);
        oracle_col_sums(n, t, x, y, hyper, lam_, n, NULL, G, H, nthreads);
        for (int64_t j = 0; j < n; ++j) {
            if (grad_theta) grad_theta[j] = G[j] - ig[11 * j + 7];
            if (negH_theta) negH_theta[j] = H[j];
        }
        free(G);
        free(H);
    }
    free(col);
    free(ig);
    free(tmp);
    free(lam_);
    free(acc);
    return 0;
}
