/*
 * sic step-level C-ABI: the individual steps of one block update of the
 * block coordinate-descent relaxation (Section 6.1, Algorithm 2) and of the
 * multilevel cycle (Section 3, Algorithm 1; Section 7), exposed so that each
 * step can be checked on its own against a reference. The solver in sic.h
 * runs exactly these steps, through the same kernels.
 *
 * All host arrays are caller-owned; sizes are given explicitly; return codes
 * are the SIC_* codes of sic.h.
 */
#ifndef SIC_STEPS_H
#define SIC_STEPS_H

#include "sic.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sic_prob sic_prob;

/* Device-resident problem state: samples X (m x n row-major float64, host or
 * device pointer, copied), lambda, and the iterate A = I. */
int sic_prob_create(sic_ctx* ctx, const double* X, int64_t n, int64_t m, double lambda,
                    sic_prob** out);
void sic_prob_destroy(sic_prob* p);

/* Replace the iterate by a host CSR (full symmetric, sorted columns). The
 * tracked objective becomes `objective` (pass NAN when unknown). */
int sic_prob_set_A(sic_prob* p, const sic_csr* A, double objective);
/* Copy the iterate out (library-allocated arrays: release with sic_csr_free). */
int sic_prob_get_A(sic_prob* p, sic_csr* out);
/* Tracked objective F(A) (changes accumulate from the line search). */
double sic_prob_objective(sic_prob* p);

/* (a) Covariance columns S_J = X^T X[:, j0:j0+b] / m (Section 6, samples
 * kept, S implicit). out: n x b row-major host array. */
int sic_step_cov_block(sic_prob* p, int64_t j0, int b, double* out);

/* (a, mixed precision) The same block from X narrowed to x_dtype (SIC_X_F32:
 * float; SIC_X_BF16: bfloat16, round to nearest even) with float
 * accumulation on the matrix cores, widened to float64. out as above.
 * SIC_EINVAL for another dtype or a bad range. */
int sic_step_cov_block_low(sic_prob* p, int64_t j0, int b, int x_dtype, double* out);

/* (a, coarse levels) Sampled covariance entries S_{r_t c_t} for `count`
 * pairs (Section 7: only entries in C_l are needed). out: count doubles. */
int sic_step_cov_pairs(sic_prob* p, const int32_t* rows, const int32_t* cols, int64_t count,
                       double* out);

/* (b) Inverse columns W_J = A^{-1} E_J by block conjugate gradients with a
 * Jacobi preconditioner (Section 6.1). cols: k column indices; out: n x k
 * row-major host array. tol: max relative residual over the columns. */
int sic_step_inverse_columns(sic_prob* p, const int32_t* cols, int k, double tol, int max_iter,
                             double* out, int* iterations, double* max_rel_residual);

/* (b) The same inverse columns for callers that cannot allocate memory
 * (code under HIP graph capture, serving loops with a fixed footprint,
 * harnesses that forbid hipMalloc): no device or host allocation happens in
 * this call. Every buffer of the solve lives in one static device array of
 * 128 MiB per GPU (held until the process ends); a solve needs about
 * 24 n k bytes (three n x k float64 arrays) plus 8 nnz + O(n + k), which
 * sic_step_inverse_columns_noalloc_limit reports (0 when it does not fit),
 * and k <= 4096. Larger problems return SIC_ETOOBIG.
 *   rowptr[n+1], col[nnz], val[nnz]: A as a full symmetric CSR with sorted
 *     columns, DEVICE memory, caller-owned, only read;
 *   cols[k]: column indices in [0, n), DEVICE memory (an index outside that
 *     range yields a zero column);
 *   W: n x k row-major, DEVICE memory, written;
 *   stream: hipStream_t on the current device (NULL: the null stream).
 * The call returns after the solve has finished on `stream`. Results equal
 * sic_step_inverse_columns' for the same A, columns and tolerance. Every
 * call on one GPU uses that GPU's array and leaves its contents behind (the
 * solve initialises all it reads): calls that overlap on one GPU, from
 * several host threads or streams, race and give wrong results. */
int sic_step_inverse_columns_noalloc(const int64_t* rowptr, const int32_t* col,
                                     const double* val, int64_t n, int64_t nnz,
                                     const int32_t* cols, int k, double tol, int max_iter,
                                     double* W, void* stream, int* iterations,
                                     double* max_rel_residual);
size_t sic_step_inverse_columns_noalloc_limit(int64_t n, int64_t nnz, int k);

/* Level set C_l for coarse block updates (Section 7, eq. (MLE_l1_prior_C)):
 * `count` pair keys i*n + j with i <= j. */
int sic_step_set_level(sic_prob* p, const int64_t* keys, int64_t count);

typedef struct {
    int64_t E;          /* free entries of the block columns (both in-block triangles) */
    int64_t n_neighbors;/* |N| (Section 6.1.1, eq. (extended_set)) */
    int64_t n_level_nbrs;/* |N^C| at a coarse level (App. A.2) */
    int64_t n_coords;   /* descent coordinates (each free pair once) */
    int cg_iterations_I, cg_iterations_N;
    int cd_sweeps;
    double cd_last_max_mu;
    double alpha;       /* step length (0 when no trial decreased F) */
    double dF;          /* F(A + alpha Delta) - F(A) */
    int trials;
    int64_t nnz_after;
} sic_block_result;

/* One complete block update on columns [j0, j0+b): level 0 is the finest
 * level; level > 0 restricts the free set to the level set given by
 * sic_step_set_level. tol_I / tol_N: CG tolerances (<= 0: defaults). */
int sic_step_block(sic_prob* p, int64_t j0, int b, int level, double tol_I, double tol_N,
                   sic_block_result* res);

/* Intermediate results of the last block update:
 *   colptr[b+1], rows[E], g[E]: free set per block column (rows ascending), gradient S - W
 *   nbrs[n_neighbors]: N ascending
 *   coord_rows[n_coords], coord_cols[n_coords], delta[n_coords]: coordinates (global
 *     indices, column-major order) and the Newton direction
 *   wjj[(b+|N|)^2]: W on J' = I u N (I first, then N), row-major
 * Any output pointer may be NULL. */
int sic_step_last_block(sic_prob* p, int64_t* colptr, int32_t* rows, double* g, int32_t* nbrs,
                        int32_t* coord_rows, int32_t* coord_cols, double* delta, double* wjj);

/* One relaxation sweep over all blocks (level 0 finest, > 0 the level set).
 * kkt_max / kkt_l1 (finest level only, may be NULL): min-norm subgradient
 * of each block measured before its update (Section 4, eq. (subgradient1)). */
int sic_step_sweep(sic_prob* p, int level, double tol_I, double tol_N, double* kkt_max,
                   double* kkt_l1);

/* Exact KKT measure of the current iterate (all blocks, CG to tol_cg). */
int sic_step_kkt(sic_prob* p, double tol_cg, double* kkt_max, double* kkt_l1);

/* Coordinate descent on given data (host arrays), the kernel of step (d):
 *   wjj: jp x jp (W on J', block columns first), cptr[b+1]: coordinates per
 *   block column, cp[n_coords]: local row index in J', S/A: per coordinate.
 * delta_out: n_coords; stats_out[7]: sweeps, last max|mu|, max|Delta|, then
 * four phase clocks of the kernel (device wall clock, 100 MHz ticks): with
 * the explicit coordinate Hessian (n_coords <= the context's cd_hessian_max)
 * the serial chain, the Hessian products, the staging waits and 0; otherwise
 * staging u, dot products and gathers, the serial chain and folding steps
 * into U. Both forms visit the coordinates in the same order. */
int sic_step_cd(sic_ctx* ctx, int jp, int b, const double* wjj, const int64_t* cptr,
                const int32_t* cp, const double* S, const double* A, double lambda,
                int max_sweeps, double tol, double* delta_out, double* stats_out);

/* Line search of step (e) on given data (same layout as sic_step_cd plus the
 * direction): returns alpha, dF and the number of trials. logdet_out
 * (optional, n_alpha entries) receives log det(A + a Delta) - log det A for
 * a = 2^-i, i < n_alpha (NaN when not PD). */
int sic_step_linesearch(sic_ctx* ctx, int jp, int b, const double* wjj, const int64_t* cptr,
                        const int32_t* cp, const double* S, const double* A, const double* delta,
                        double lambda, double* alpha, double* dF, int* trials,
                        double* logdet_out, int n_alpha);

/* Multilevel hierarchy (Section 3.2, Section 7): ranking of the pair keys
 * (support first, then free pairs by |g| descending, ties by key) and the
 * level sizes |C_1| >= ... >= |C_L| = |supp|. ranking_out: capacity
 * n_supp + n_free; sizes_out: capacity 64. */
int sic_hierarchy(int64_t n, const int64_t* supp_keys, int64_t n_supp, const int64_t* free_keys,
                  const double* free_absg, int64_t n_free, int64_t* ranking_out,
                  int64_t* ranking_len, int64_t* sizes_out, int* n_levels);

/* Clustered block partition (Section 6.1; eq. (extended_set) of Section
 * 6.1.1: blocks whose free pairs stay inside them have small neighbourhoods
 * N_j). The graph has a vertex per variable and an edge per pair key
 * i*n + j (diagonal keys and repeats ignored). Blocks of b vertices are grown
 * one after another, breadth-first from a seed over unplaced vertices
 * (neighbours in ascending order); a growth that exhausts its component goes
 * on from the next seed. The next seed is the oldest unplaced candidate
 * (vertices adjacent to earlier blocks, queued when each block was completed:
 * members in order, each one's neighbours ascending), else the unplaced
 * vertex of least degree (ties: smaller index). order_out[n] (caller-owned)
 * receives the variables in block order: block k is order_out[k b .. k b + b).
 * Host computation only. SIC_EINVAL for bad sizes or keys outside [0, n^2). */
int sic_cluster_order(int64_t n, const int64_t* keys, int64_t count, int b, int32_t* order_out);

#ifdef __cplusplus
}
#endif
#endif /* SIC_STEPS_H */
