/*
 * fd_oracle.c -- plain FP64 reference stepper for the second-order acoustic
 * wave equation (test infrastructure, not part of the product).
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code, header, table or
 * helper with the GPU library; the arrays it receives are computed by the
 * Python side of the oracle (oracle/__init__.py) from the same readings.
 *
 * What it computes (the thesis benchmarks a finite-difference stepper built
 * from a Grid, a TimeFunction of given time/space order, Functions for the
 * medium and SparseTimeFunctions for sources and receivers, advanced by an
 * Operator called with a number of time steps -- Section 2.1.1; the acoustic
 * problem with sources and receivers is the case named in Section 6.2.1):
 *
 *   m u_tt + m sigma u_t - Lap_h u = q         (m = 1/v^2)
 *
 * discretised with central differences in time (leapfrog, damping term
 * centred) and the maximal-order central second-derivative stencil in each
 * axis (the star stencil of Section 3.3.3, "Stencil creation"), with the
 * field taken as zero outside the padded grid.  Every loop below is the
 * plain definition: one pass over all points per time step, no blocking,
 * no fusion, no reordering.
 *
 * Array conventions: a field is a dense C array over the padded grid with
 * axis 0 (x) fastest: index = i0 + n0*(i1 + n1*i2).  ndim is 2 or 3.
 */
#include <stdlib.h>
#include <string.h>

#define MAXR 8

static long total_points(int ndim, const long *n)
{
    long t = 1;
    for (int a = 0; a < ndim; ++a) t *= n[a];
    return t;
}

/*
 * Discrete Laplacian, O4: out_i = sum_a h_a^-2 [c_0 u_i + sum_j c_j (u_{i+j e_a} + u_{i-j e_a})]
 * with u = 0 outside the grid.  c[0..r] are the second-derivative weights.
 */
void orc_laplacian(int ndim, const long *n, const double *h, int r,
                   const double *c, const double *u, double *out)
{
    /* a 2D grid is handled as a 3D grid with a single plane along axis 2 */
    const long n0 = n[0], n1 = n[1], n2 = (ndim == 3) ? n[2] : 1;
    const long stride[3] = {1, n0, n0 * n1};
    double ih2[3] = {0.0, 0.0, 0.0};
    for (int a = 0; a < ndim; ++a) ih2[a] = 1.0 / (h[a] * h[a]);
#pragma omp parallel for schedule(static)
    for (long i2 = 0; i2 < n2; ++i2) {
        for (long i1 = 0; i1 < n1; ++i1) {
            for (long i0 = 0; i0 < n0; ++i0) {
                const long idx[3] = {i0, i1, i2};
                const long i = i0 + n0 * (i1 + n1 * i2);
                double acc = 0.0;
                for (int a = 0; a < ndim; ++a) {
                    const long na = (a == 0) ? n0 : (a == 1) ? n1 : n2;
                    double s = c[0] * u[i];
                    for (int j = 1; j <= r; ++j) {
                        double up = (idx[a] + j < na) ? u[i + j * stride[a]] : 0.0;
                        double dn = (idx[a] - j >= 0) ? u[i - j * stride[a]] : 0.0;
                        s += c[j] * (up + dn);
                    }
                    acc += ih2[a] * s;
                }
                out[i] = acc;
            }
        }
    }
}

/*
 * One leapfrog step, O6:
 *   u_next = [2 u - (1 - sigma dt/2) u_prev + dt^2 v^2 (lap + q)] / (1 + sigma dt/2)
 * lap is Lap_h u (precomputed), q the source density (may be NULL = 0).
 */
static void leapfrog(long tot, double dt, const double *vel, const double *sigma,
                     const double *u, const double *u_prev, const double *lap,
                     const double *q, double *u_next)
{
#pragma omp parallel for schedule(static)
    for (long i = 0; i < tot; ++i) {
        double s = sigma[i] * dt / 2.0;
        double src = q ? q[i] : 0.0;
        double rhs = 2.0 * u[i] - (1.0 - s) * u_prev[i]
                   + dt * dt * vel[i] * vel[i] * (lap[i] + src);
        u_next[i] = rhs / (1.0 + s);
    }
}

/*
 * Forward modelling, O6 + O8 + O9.
 *   nc grid points per sparse point (2^ndim multilinear corners, or (2r)^ndim
 *   windowed-sinc nodes); src_idx/src_w are [nsrc][nc] (flat padded index,
 *   weight; weight 0 for nodes dropped outside the grid), rec_idx/rec_w
 *   likewise.
 *   wavelet is [nt][nsrc]; sample n enters u^{n+1} as
 *   q = sum_s w_s[n] W_s / prod(h)   (discrete delta, O8).
 *   rec[n][r] = sum_c W_{r,c} u^{n+1}[idx_{r,c}]   (O9), n = 0..nt-1.
 *   u_cur / u_prev: on entry u^0 and u^{-1}; on exit u^{nt} and u^{nt-1}.
 *   history (nullable): (nt+2) fields u^{-1}, u^0, ..., u^{nt}.
 * Returns 0, or -1 on allocation failure.
 */
int orc_forward(int ndim, const long *n, const double *h, int r, const double *c,
                const double *vel, const double *sigma, double dt, int nt,
                int nc, int nsrc, const long *src_idx, const double *src_w, const double *wavelet,
                int nrec, const long *rec_idx, const double *rec_w, double *rec,
                double *u_cur, double *u_prev, double *history)
{
    const long tot = total_points(ndim, n);
    double cell = 1.0;
    for (int a = 0; a < ndim; ++a) cell *= h[a];

    double *lap = malloc(sizeof(double) * tot);
    double *q = calloc(tot, sizeof(double));
    double *u_next = malloc(sizeof(double) * tot);
    if (!lap || !q || !u_next) {
        free(lap); free(q); free(u_next);
        return -1;
    }
    double *a = u_cur, *b = u_prev;   /* a = u^n, b = u^{n-1} */
    if (history) {
        memcpy(history, b, sizeof(double) * tot);
        memcpy(history + tot, a, sizeof(double) * tot);
    }
    for (int t = 0; t < nt; ++t) {
        for (int s = 0; s < nsrc; ++s)
            for (int k = 0; k < nc; ++k)
                q[src_idx[s * nc + k]] += wavelet[(long)t * nsrc + s] * src_w[s * nc + k] / cell;
        orc_laplacian(ndim, n, h, r, c, a, lap);
        leapfrog(tot, dt, vel, sigma, a, b, lap, q, u_next);
        for (int s = 0; s < nsrc; ++s)
            for (int k = 0; k < nc; ++k)
                q[src_idx[s * nc + k]] = 0.0;
        for (int rr = 0; rr < nrec; ++rr) {
            double v = 0.0;
            for (int k = 0; k < nc; ++k)
                v += rec_w[rr * nc + k] * u_next[rec_idx[rr * nc + k]];
            rec[(long)t * nrec + rr] = v;
        }
        /* rotate: u^{n-1} <- u^n, u^n <- u^{n+1} */
        memcpy(b, a, sizeof(double) * tot);
        memcpy(a, u_next, sizeof(double) * tot);
        if (history) memcpy(history + (long)(t + 2) * tot, a, sizeof(double) * tot);
    }
    free(lap); free(q); free(u_next);
    return 0;
}

/*
 * Adjoint modelling, O11 (the exact transpose of orc_forward for fixed v):
 *   lam^{nt} = lam^{nt+1} = 0; for k = nt..1:
 *   lam^{k-1} = [2 lam^k - (1 - sigma dt/2) lam^{k+1} + dt^2 v^2 Lap_h lam^k
 *                + v^2 sum_r W_r res_r[k-1]] / (1 + sigma dt/2)
 *   out[n][s] = dt^2 / prod(h) * sum_c W_{s,c} lam^n[idx_{s,c}]
 * lam_hist (nullable) receives nt fields lam^0 .. lam^{nt-1}.
 */
int orc_adjoint(int ndim, const long *n, const double *h, int r, const double *c,
                const double *vel, const double *sigma, double dt, int nt,
                int nc, int nsrc, const long *src_idx, const double *src_w, double *src_out,
                int nrec, const long *rec_idx, const double *rec_w, const double *residual,
                double *lam_hist)
{
    const long tot = total_points(ndim, n);
    double cell = 1.0;
    for (int a = 0; a < ndim; ++a) cell *= h[a];

    double *lap = malloc(sizeof(double) * tot);
    double *q = calloc(tot, sizeof(double));
    double *la = calloc(tot, sizeof(double));   /* lam^k */
    double *lb = calloc(tot, sizeof(double));   /* lam^{k+1} */
    double *lnew = malloc(sizeof(double) * tot);
    if (!lap || !q || !la || !lb || !lnew) {
        free(lap); free(q); free(la); free(lb); free(lnew);
        return -1;
    }
    for (int k = nt; k >= 1; --k) {
        /* the receiver term enters as v^2 P_r^T r; written as dt^2 v^2 (q)
           with q = P_r^T r / dt^2 so that the shared leapfrog applies */
        for (int rr = 0; rr < nrec; ++rr)
            for (int j = 0; j < nc; ++j)
                q[rec_idx[rr * nc + j]] += residual[(long)(k - 1) * nrec + rr] * rec_w[rr * nc + j] / (dt * dt);
        orc_laplacian(ndim, n, h, r, c, la, lap);
        leapfrog(tot, dt, vel, sigma, la, lb, lap, q, lnew);
        for (int rr = 0; rr < nrec; ++rr)
            for (int j = 0; j < nc; ++j)
                q[rec_idx[rr * nc + j]] = 0.0;
        for (int s = 0; s < nsrc; ++s) {
            double v = 0.0;
            for (int j = 0; j < nc; ++j)
                v += src_w[s * nc + j] * lnew[src_idx[s * nc + j]];
            src_out[(long)(k - 1) * nsrc + s] = dt * dt / cell * v;
        }
        if (lam_hist) memcpy(lam_hist + (long)(k - 1) * tot, lnew, sizeof(double) * tot);
        memcpy(lb, la, sizeof(double) * tot);
        memcpy(la, lnew, sizeof(double) * tot);
    }
    free(lap); free(q); free(la); free(lb); free(lnew);
    return 0;
}

/*
 * Imaging condition, O12: given the forward history u^{-1}..u^{nt}
 * ((nt+2) fields) and the adjoint fields lam^0..lam^{nt-1} driven by the
 * residual, accumulate
 *   g_i = - sum_{n=0}^{nt-1} lam^n_i [(u^{n+1} - 2u^n + u^{n-1})_i
 *                                     + (sigma_i dt/2)(u^{n+1} - u^{n-1})_i]
 */
void orc_imaging(int ndim, const long *n, const double *sigma, double dt, int nt,
                 const double *history, const double *lam_hist, double *grad)
{
    const long tot = total_points(ndim, n);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < tot; ++i) {
        double g = 0.0;
        double s = sigma[i] * dt / 2.0;
        for (int t = 0; t < nt; ++t) {
            double um = history[(long)t * tot + i];         /* u^{t-1} */
            double u0 = history[(long)(t + 1) * tot + i];   /* u^t     */
            double up = history[(long)(t + 2) * tot + i];   /* u^{t+1} */
            g -= lam_hist[(long)t * tot + i] * ((up - 2.0 * u0 + um) + s * (up - um));
        }
        grad[i] = g;
    }
}

/* Threads for the loops above from now on (n >= 1; the CPU baseline times
   the oracle on one core as well as on all of them). */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    extern void omp_set_num_threads(int);
    if (n >= 1) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* OpenMP thread count actually used by the loops above (for reporting). */
int orc_num_threads(void)
{
    int nth = 1;
#pragma omp parallel
    {
#pragma omp single
        {
#ifdef _OPENMP
            extern int omp_get_num_threads(void);
            nth = omp_get_num_threads();
#endif
        }
    }
    return nth;
}
