/*
 * sic profiling C-ABI: optional per-kernel timing with HIP events on the
 * stream each kernel is launched on, plus the algorithmic bytes and flops of
 * every timed launch (the traffic and work the kernel must do at minimum), so
 * that achieved bandwidth / throughput can be reported without a profiler.
 * Timing adds two event records per launch; leave it off for production runs.
 * The switch, the class selection and the counters belong to the calling host
 * thread: a solve is timed on the thread that runs it.
 */
#ifndef SIC_PROFILE_H
#define SIC_PROFILE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Kernel classes:
 *   0 sj_gemm_f64  covariance columns (MFMA)     5 cd           coordinate descent
 *   1 sddmm        sampled covariance entries    6 chol         line-search Cholesky
 *   2 cg_spmm      CG sparse product             7 gemm_small   line-search products
 *   3 cg_update    CG vector update              8 upd_rows     CSR rebuild
 *   4 screen_fine  free-set screening            9 cd_hess      coordinate Hessian
 *                                                               (explicit-Hessian CD)
 *                                               10 trsm         triangular solves
 *                                               11 pcd          PCD-CG Newton direction
 *                                               12 sj_gemm_f32  S_J from float X (mixed precision)
 *                                               13 sj_gemm_bf16 S_J from bfloat16 X (mixed precision) */
#define SIC_KERNEL_CLASSES 14

void sic_profile_enable(int on);      /* on != 0 starts timing, 0 stops it */
void sic_profile_reset(void);         /* zero every counter */
/* Restrict timing to the classes whose bit (1 << class) is set in mask; the
 * others launch with no event around them. The default selects every class. */
void sic_profile_select(uint32_t mask);
/* Totals of one kernel class since the last reset; returns SIC_EINVAL (-1)
 * for an unknown class. Any output pointer may be NULL. */
int sic_profile_read(int kind, int64_t* launches, double* milliseconds, double* bytes,
                     double* flops);
const char* sic_profile_kernel_name(int kind);

#ifdef __cplusplus
}
#endif
#endif /* SIC_PROFILE_H */
