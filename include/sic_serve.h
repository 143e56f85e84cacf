/*
 * sic — serving loop: continuous batching of estimation problems on one GPU.
 *
 * A server owns `slots` solver contexts. Each slot is one solver context (a
 * non-blocking HIP stream and the context's second stream, and its own device
 * workspace), driven by one host worker thread.
 * Submitted problems wait in a FIFO queue. A problem is admitted when a slot
 * is idle and its device-memory footprint fits in what the admitted problems
 * leave of the server's budget. Problems that arrive while others run are
 * admitted as soon as a slot and memory free up. The block updates of all
 * admitted problems (Algorithm 2, Section 6.1, inside the cycles of
 * Algorithm 1) then run concurrently on the device, on each problem's streams,
 * and each problem's X, iterate A, level sets and workspace stay resident on
 * the device until it finishes.
 *
 * A problem is a sic_problem (sic.h): one lambda, or a decreasing lambda path
 * solved in order within one request, each result warm-starting the next.
 * Every result is the one that
 * sic_solve_batch gives for the same problem and options: the kernels and
 * their order within a problem do not depend on what else runs.
 *
 * Ownership: the server copies lambda_path and A0 at submission, but reads
 * problem->X (host or device memory) when the request is admitted: the caller
 * keeps X valid and unchanged until sic_server_wait has returned the request
 * (or it was cancelled).
 * Results are host CSR arrays allocated by the library (release each with
 * sic_csr_free).
 *
 * Thread safety: every sic_server_* call may be made from any host thread.
 */
#ifndef SIC_SERVE_H
#define SIC_SERVE_H

#include "sic.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct sic_server sic_server;

typedef struct {
    int slots;            /* problems solved concurrently, 1..64; 0 = 4 */
    size_t hbm_budget;    /* device bytes all admitted problems may hold together;
                             0 = 80% of the device memory free at creation */
    sic_options solver;   /* per-problem solver options; device, stream and trace are
                             ignored (the server uses opt.device of sic_server_create) */
    int device;           /* HIP device ordinal */
} sic_server_options;

/* Per-request timing, in seconds since the server was created. */
typedef struct {
    double submitted, admitted, finished;
    size_t footprint;     /* the admission estimate, bytes */
    int slot;             /* the slot that ran it, or -1 */
} sic_request_times;

/* Fill *opt with defaults (4 slots, budget 0 = 80% of free memory, solver defaults). */
void sic_server_options_default(sic_server_options* opt);

/* Create a server and start its worker threads. */
int sic_server_create(sic_server** out, const sic_server_options* opt);

/* Device bytes the server would reserve for problem p (the admission estimate):
 * X and its transpose in float64, the iterate's CSR at up to n^2 entries, and
 * the block workspace at its largest (block CG on all n columns, dense W on
 * the neighbourhood, coordinate Hessian). Returns 0 for an invalid problem. */
size_t sic_server_footprint(const sic_server* srv, const sic_problem* p);

/* Queue one problem. *ticket receives its id. SIC_ENOMEM if its footprint alone
 * exceeds the server's budget, SIC_EINVAL for bad arguments, SIC_ECANCELED
 * after shutdown began. */
int sic_server_submit(sic_server* srv, const sic_problem* p, uint64_t* ticket);

/* Wait until request `ticket` completes, at most timeout_s seconds (< 0: no
 * limit). On completion its results are moved to A_out / info (arrays of
 * sic_request_results(p) slots, as in sic_solve_batch; either may be NULL to
 * drop them) and the ticket is retired: the return value is the request's
 * status. Returns 1 (and keeps the ticket) on timeout, SIC_EINVAL for an
 * unknown ticket. */
int sic_server_wait(sic_server* srv, uint64_t ticket, double timeout_s, sic_csr* A_out,
                    sic_info* info, sic_request_times* times);

/* Cancel a request that has not been admitted yet (its wait then returns
 * SIC_ECANCELED). Returns SIC_OK, or SIC_EINVAL if it is unknown, running or
 * done. */
int sic_server_cancel(sic_server* srv, uint64_t ticket);

/* Number of results a problem produces (n_lambda, or 1). */
int sic_request_results(const sic_problem* p);

/* Snapshot: queued, running and finished-but-unclaimed requests, and device
 * bytes the slots hold now. Any pointer may be NULL. */
void sic_server_status(const sic_server* srv, int* queued, int* running, int* done,
                       size_t* held_bytes);

/* Cancel what is queued, finish what runs, join the workers, free everything
 * (unclaimed results included). NULL is allowed. */
void sic_server_destroy(sic_server* srv);

#ifdef __cplusplus
}
#endif
#endif /* SIC_SERVE_H */
