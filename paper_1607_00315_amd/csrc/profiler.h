// Optional per-kernel timing (see profiler.hip).
#pragma once

#include "sic_internal.h"

namespace sic {

enum KernelKind {
    KK_SJ = 0,
    KK_SDDMM,
    KK_CG_SPMM,
    KK_CG_UPDATE,
    KK_SCREEN,
    KK_CD,
    KK_CHOL,
    KK_GEMM,
    KK_UPD_ROWS,
    KK_CD_HESS,
    KK_TRSM,
    KK_PCD,
    KK_SJ_F32,
    KK_SJ_BF16,
    KK_COUNT
};

struct KernelStat {
    int64_t launches = 0;
    double ms = 0, bytes = 0, flops = 0;
};

const char* kernel_kind_name(int kind);
void prof_enable(bool on);
bool prof_enabled();
void prof_reset();
void prof_begin(int kind, hipStream_t s);
// returns a handle usable with prof_discard until the next prof_flush
int64_t prof_end(int kind, hipStream_t s, double bytes, double flops);
void prof_discard(int64_t handle);
void prof_scale(int64_t handle, double factor);
void prof_flush();
KernelStat prof_read(int kind);

}  // namespace sic
