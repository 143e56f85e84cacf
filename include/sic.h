/*
 * sic — sparse inverse covariance estimation on AMD Instinct MI355X (gfx950).
 *
 * Public C-ABI of the solver for the l1-regularised Gaussian maximum-likelihood
 * problem (Treister, Turek, Yavneh: "A multilevel framework for sparse
 * optimization with application to inverse covariance estimation and logistic
 * regression", Section 5, eq. (MLE_l1_prior)):
 *
 *     minimise over A > 0:   F(A) = -log det A + tr(S A) + lambda * sum_ij |A_ij|
 *
 * with S = X^T X / m formed only implicitly from the m x n sample matrix X
 * (the samples are kept, S is never stored: Section 5, Section 6).
 * The solver is the multilevel cycle of Algorithm 1 (Section 3.1, Section 7)
 * over the block coordinate-descent relaxation of Algorithm 2 (Section 6.1):
 * every block update computes the covariance columns S_J, the inverse columns
 * W_J = A^{-1} E_J by block conjugate gradients, the free set, a coordinate-
 * descent Newton direction and a positive-definite line search through the
 * Schur complement (Section 6.1.2, App. A.1), all as HIP kernels on the GPU.
 *
 * Conventions shared by every entry point:
 *   - Matrices of samples are m x n ROW-MAJOR (row = one sample).
 *   - Sparse results are full symmetric CSR (both triangles) with int64 row
 *     pointers, int32 column indices sorted ascending within each row, and
 *     float64 values.
 *   - Every function returns SIC_OK (0) or a negative error code below;
 *     sic_strerror() names it and sic_last_error() gives the last message of
 *     the calling thread.
 *   - A context is not thread-safe: use one context per host thread.
 */
#ifndef SIC_H
#define SIC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ codes */
#define SIC_OK 0
#define SIC_EINVAL -1      /* bad argument: n < 1, m < 1, lambda < 0, tol <= 0, NULL pointer,
                              lambda = 0 with m <= n (S singular: no estimate, Section 5) */
#define SIC_ENONFINITE -2  /* non-finite value in X or in a warm start */
#define SIC_ENOTPD -3      /* warm start not positive definite (the line search needs a PD
                              start, Section 6.1.2) */
#define SIC_ENOMEM -4      /* device allocation failed or the footprint exceeds hbm_budget */
#define SIC_ENOCONV -5     /* max_cycles reached before tol; outputs are still filled */
#define SIC_EHIP -6        /* HIP runtime error */
#define SIC_ECANCELED -7   /* request cancelled (serving) */
#define SIC_ETOOBIG -8     /* a block working set exceeds a kernel's static limit */
#define SIC_EINTERNAL -9   /* internal consistency check failed */

/* precision modes */
#define SIC_FP64 0         /* every step in float64 */
#define SIC_MIXED 1        /* reduced-precision S_J / CG while far from the optimum */

/* sample dtypes for sic_problem.x_dtype */
#define SIC_X_F64 0
#define SIC_X_F32 1
#define SIC_X_BF16 2

/* option flags */
#define SIC_FLAG_NO_MULTILEVEL (1ull << 0) /* plain block relaxation (Algorithm 2 only) */
#define SIC_FLAG_FINAL_KKT (1ull << 1)     /* also measure the exact KKT of an unconverged result */
#define SIC_FLAG_VERBOSE (1ull << 2)       /* per-cycle log on stderr */
#define SIC_FLAG_NO_CERTIFY (1ull << 3)    /* accept the sweep's KKT measure without the exact
                                              float64 pass (see sic_solve) */
#define SIC_FLAG_CLUSTER (1ull << 4)       /* blocks from a clustering of the free-set graph
                                              (Section 6.1): at the start of every cycle the
                                              variables are relabelled so that each block of b
                                              consecutive ones is a breadth-first-grown cluster
                                              of the graph of A's support and the last finest
                                              sweep's free pairs (sic_cluster_order); results
                                              come back in the caller's labels */
#define SIC_FLAG_NO_WARM_CG (1ull << 6)    /* start every conjugate-gradient solve from zero.
                                              By default, a problem whose n^2 doubles fit in
                                              2 GiB keeps the inverse columns it has solved
                                              (n^2 doubles of device memory) and starts each
                                              solve from the latest ones */
#define SIC_FLAG_NO_S_CACHE (1ull << 7)    /* compute S_J = X^T X_J / m afresh for every block.
                                              By default, a problem whose n^2 doubles fit in
                                              2 GiB keeps the float64 columns of S it has formed
                                              (n^2 doubles of device memory) and copies them out
                                              in later cycles (the same values: only the time
                                              differs); with SIC_MIXED the columns are then
                                              float64 in every cycle, and the bfloat16 and float
                                              products of S_J run only with this flag */
#define SIC_FLAG_CONTINUATION (1ull << 5)  /* continuation (the BCDcont schedule of Section 8):
                                              the first three cycles run at lambda_4 =
                                              (1 + lambda) / 2 and then two values linearly
                                              spaced down towards lambda, one cycle each; the
                                              fourth and later cycles run at lambda. With
                                              SIC_FLAG_NO_MULTILEVEL this is BCDcont */

typedef struct sic_ctx sic_ctx;

typedef struct {
    int64_t n, nnz;
    int64_t* rowptr; /* [n+1] */
    int32_t* col;    /* [nnz] */
    double* val;     /* [nnz] */
} sic_csr;

typedef struct {
    double seconds;    /* since the start of the solve */
    double objective;  /* tracked F(A) after the cycle */
    double kkt_max;    /* finest sweep's max-norm of the min-norm subgradient */
    double kkt_rel_l1; /* its l1 norm over ||A||_1 (the stopping measure of Section 8) */
    int64_t nnz;       /* non-zeros of A (both triangles) */
    int32_t cycle;
    int32_t levels;    /* coarse levels visited in this cycle */
} sic_trace_entry;

typedef struct {
    int device;            /* HIP device ordinal */
    size_t hbm_budget;     /* bytes the context may allocate (0 = no limit) */
    int precision;         /* SIC_FP64 or SIC_MIXED */
    int block;             /* block size b (columns per block), default 256 */
    double cg_tol_I;       /* relative CG residual for W_I, default 1e-5 (Section 8) */
    double cg_tol_N;       /* relative CG residual for W_N, default 1e-4 (Section 8) */
    int cg_max_iter;       /* CG iteration cap per solve, default 1000 */
    double cd_tol;         /* CD stop: max|mu| <= cd_tol * max|Delta|, default 1e-4 */
    int cd_max_sweeps;     /* CD sweep cap per block, default 20 */
    int cd_hessian_max;    /* blocks with at most this many coordinates run CD on an explicit
                              coordinate Hessian (ncoord^2 doubles of scratch); 0 = default
                              4096, < 0 = never */
    int pcd_min_coords;    /* blocks with at least this many coordinates take the Newton
                              direction by PCD-CG (Section 6.1.1) instead of the sequential
                              coordinate chain; 0 = default 4097, < 0 = never */
    int ls_max_trials;     /* line-search trials alpha = 2^-i, i < ls_max_trials, default 31 */
    int max_cycles;        /* multilevel cycles, default 100 */
    void* stream;          /* hipStream_t to run on, or NULL for the context's own stream */
    uint64_t flags;        /* SIC_FLAG_* */
    sic_trace_entry* trace;/* optional per-cycle trace (caller-owned), may be NULL */
    int trace_cap;
} sic_options;

typedef struct {
    double objective;   /* F(A) tracked through the line-search changes */
    double kkt_max;     /* last finest sweep's max |min-norm subgradient| (or the exact pass) */
    double kkt_rel_l1;  /* ||min-norm subgradient||_1 / ||A||_1 (the paper's stopping measure) */
    int64_t nnz, max_nnz;
    int cycles, sweeps;
    int64_t blocks, cg_iterations, cd_sweeps;
    double seconds;
    int status;
    int trace_len;
} sic_info;

typedef struct {
    const void* X;          /* m x n row-major samples, host or device memory */
    int64_t n, m;
    int x_dtype;            /* SIC_X_F64 / SIC_X_F32 / SIC_X_BF16 */
    double lambda;          /* used when n_lambda == 0 */
    double tol;             /* KKT max-norm target */
    const sic_csr* A0;      /* optional PD warm start (host CSR), may be NULL */
    const double* lambda_path; /* optional decreasing lambdas solved in order, warm-started */
    int n_lambda;
} sic_problem;

/* Fill *opt with the defaults listed above. */
void sic_options_default(sic_options* opt);

/* Create a context on opt->device (opt may be NULL for defaults). */
int sic_create(sic_ctx** out, const sic_options* opt);

/* Destroy a context and every device buffer it owns. NULL is allowed. */
void sic_destroy(sic_ctx* ctx);

/*
 * Solve one problem (Sections 5-7). X: m x n row-major float64, host or device
 * pointer (detected; never freed). lambda >= 0, tol > 0 is the KKT max-norm
 * target. A_out receives a host CSR allocated by the library (release it with
 * sic_csr_free); info (may be NULL) receives statistics. Returns SIC_OK,
 * SIC_ENOCONV (A_out and info still filled) or an error code. The context
 * keeps the problem's device storage (X, its copies, the CSR pair) for the
 * next solve or batch on it; sic_destroy frees it, and so does a failed solve.
 *
 * Convergence: each finest sweep measures the min-norm subgradient (Section
 * 4, eq. (subgradient1)) of every block just before its update, from the
 * sweep's own S_J and W_J. When that measure reaches tol in a float64 cycle,
 * an exact pass recomputes it for the final iterate (float64 S_J, W_J by CG to
 * min(1e-10, 0.01 tol)) and SIC_OK is returned only if that too is <= tol;
 * info->kkt_max is then the exact value. Otherwise the cycles go on. If a
 * conjugate-gradient solve stops at cg_max_iter, the block it served is left
 * unchanged and the solve ends with SIC_ENOCONV (the iterate returned is the
 * last accepted one); a CG breakdown (p.Ap <= 0) ends it with SIC_ENOTPD.
 */
int sic_solve(sic_ctx* ctx, const double* X, int64_t n, int64_t m, double lambda, double tol,
              sic_csr* A_out, sic_info* info);

/*
 * Solve several problems; problems with a lambda_path produce n_lambda results
 * each (warm-started from the previous lambda). A_out and info are arrays with
 * one slot per result, in order; each slot's status is in info[k].status.
 * Returns SIC_OK when every result converged, else the first failing status.
 */
int sic_solve_batch(sic_ctx* ctx, int count, const sic_problem* problems, sic_csr* A_out,
                    sic_info* info);

/* Release arrays the library allocated in *a and zero it. */
void sic_csr_free(sic_csr* a);

const char* sic_strerror(int code);
const char* sic_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* SIC_H */
