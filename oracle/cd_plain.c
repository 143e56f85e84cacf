/*
 * Oracle (test infrastructure only): plain cyclic coordinate descent on the
 * l1-regularised quadratic model of the log-det objective (the Newton
 * direction subproblem, Section 5.1, eq. (Quad_MLE_l1_prior), restricted to a
 * free set as in Section 5.2 / Section 6.1).
 *
 * Only the tests, the package smoke check and the benchmark's CPU-baseline leg
 * may load this file's library; the GPU library never links it.
 *
 * For one symmetric pair (i,k) the model restricted to Delta_ik = Delta_ki is
 * the 1-D problem 0.5*a*mu^2 + b*mu + lam*|c + mu| with
 *     a = W_ik^2 + W_ii*W_kk   (a = W_ii^2 when i == k)
 *     b = S_ik - W_ik + (W Delta W)_ik
 *     c = A_ik + Delta_ik
 * whose minimiser is mu = -c + soft(c - b/a, lam/a) (Section 3.2, eq. (1d_l1),
 * with the sign the minimisation gives: the printed closed form drops the
 * leading minus).
 *
 * (W Delta W)_ik is kept as the plain product through U = Delta W, stored as
 * a dense nj x nj matrix and updated by two row axpys per coordinate step.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

static double soft(double z, double t)
{
    if (z > t) return z - t;
    if (z < -t) return z + t;
    return 0.0;
}

/*
 * nj          size of the local index set J (W is nj x nj, row-major, symmetric)
 * ncoord      number of coordinates; coordinate t is the pair (ri[t], ci[t])
 * S, A        per-coordinate S_ik and A_ik
 * lam         l1 weight
 * max_sweeps  sweep cap; tol: stop after a sweep with max|mu| <= tol*max|Delta|
 * D           in/out: per-coordinate Delta (read as the starting point)
 * U           workspace of nj*nj doubles
 * verbose     nonzero: one progress line per sweep on stderr (no effect on the result)
 * returns the number of sweeps run; *last_max_mu gets the last sweep's max|mu|
 */
int oracle_cd_sweeps(int nj, const double *W, int ncoord, const int *ri, const int *ci,
                     const double *S, const double *A, double lam, int max_sweeps,
                     double tol, double *D, double *U, double *last_max_mu, int verbose)
{
    const size_t N = (size_t)nj;
    memset(U, 0, sizeof(double) * N * N);
    /* U = Delta W for the starting Delta */
    for (int t = 0; t < ncoord; ++t) {
        double d = D[t];
        if (d == 0.0) continue;
        int i = ri[t], k = ci[t];
        for (size_t p = 0; p < N; ++p) U[i * N + p] += d * W[k * N + p];
        if (i != k)
            for (size_t p = 0; p < N; ++p) U[k * N + p] += d * W[i * N + p];
    }
    int sweeps = 0;
    double maxmu = 0.0;
    for (int s = 0; s < max_sweeps; ++s) {
        maxmu = 0.0;
        for (int t = 0; t < ncoord; ++t) {
            int i = ri[t], k = ci[t];
            double wik = W[(size_t)i * N + k];
            double wii = W[(size_t)i * N + i];
            double wkk = W[(size_t)k * N + k];
            double a = (i == k) ? wii * wii : wik * wik + wii * wkk;
            double wdw = 0.0;
            for (size_t p = 0; p < N; ++p) wdw += W[(size_t)i * N + p] * U[p * N + k];
            double b = S[t] - wik + wdw;
            double c = A[t] + D[t];
            double mu = -c + soft(c - b / a, lam / a);
            if (mu != 0.0) {
                D[t] += mu;
                for (size_t p = 0; p < N; ++p) U[(size_t)i * N + p] += mu * W[(size_t)k * N + p];
                if (i != k)
                    for (size_t p = 0; p < N; ++p) U[(size_t)k * N + p] += mu * W[(size_t)i * N + p];
            }
            if (fabs(mu) > maxmu) maxmu = fabs(mu);
        }
        ++sweeps;
        double maxd = 0.0;
        for (int t = 0; t < ncoord; ++t)
            if (fabs(D[t]) > maxd) maxd = fabs(D[t]);
        if (verbose) {
            fprintf(stderr, "[oracle-cd] sweep %d of %d coordinates: max|mu| %.3e, max|Delta| %.3e\n",
                    sweeps, ncoord, maxmu, maxd);
            fflush(stderr);
        }
        if (maxmu <= tol * maxd) break;
    }
    if (last_max_mu) *last_max_mu = maxmu;
    return sweeps;
}
