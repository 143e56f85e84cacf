// Optional per-kernel timing with HIP events on the launching stream.
// Each profiled launch is bracketed by two events; the algorithmic bytes and
// flops of the launch (what the kernel must move / compute at minimum) are
// accumulated beside the measured duration, so achieved bandwidth and
// throughput follow without a profiler.
#include "profiler.h"
#include "sic_profile.h"

#include <vector>

namespace sic {

namespace {

struct Pending {
    int kind;   // -1: discarded (the launch found nothing to do)
    hipEvent_t e0, e1;
    double bytes, flops;
};

struct Profiler {
    bool enabled = false;
    uint32_t mask = ~0u;   // classes timed while enabled
    std::vector<hipEvent_t> free_events;
    std::vector<Pending> pending;
    KernelStat stat[KK_COUNT];
    hipEvent_t open[KK_COUNT] = {};
};

// Per host thread: a solve is timed on the thread that runs it, and the
// serving loop's worker threads never contend for it.
thread_local Profiler g;

hipEvent_t take_event() {
    if (!g.free_events.empty()) {
        hipEvent_t e = g.free_events.back();
        g.free_events.pop_back();
        return e;
    }
    hipEvent_t e;
    SIC_HIP(hipEventCreate(&e));
    return e;
}

void resolve() {
    if (g.pending.empty()) return;
    for (Pending& p : g.pending) {
        // launches on two streams: each record's own end event
        SIC_HIP(hipEventSynchronize(p.e1));
        if (p.kind >= 0) {
            float ms = 0.f;
            SIC_HIP(hipEventElapsedTime(&ms, p.e0, p.e1));
            KernelStat& s = g.stat[p.kind];
            s.launches += 1;
            s.ms += ms;
            s.bytes += p.bytes;
            s.flops += p.flops;
        }
        g.free_events.push_back(p.e0);
        g.free_events.push_back(p.e1);
    }
    g.pending.clear();
}

}  // namespace

const char* kernel_kind_name(int kind) {
    static const char* names[KK_COUNT] = {"sj_gemm_f64", "sddmm", "cg_spmm", "cg_update",
                                          "screen_fine", "cd", "chol", "gemm_small", "upd_rows", "cd_hess",
                                          "trsm", "pcd", "sj_gemm_f32", "sj_gemm_bf16"};
    return (kind >= 0 && kind < KK_COUNT) ? names[kind] : "?";
}

void prof_enable(bool on) {
    if (!on) resolve();
    g.enabled = on;
}

bool prof_enabled() { return g.enabled; }

void prof_reset() {
    resolve();
    for (auto& s : g.stat) s = KernelStat{};
}

void prof_begin(int kind, hipStream_t s) {
    if (!g.enabled || !((g.mask >> kind) & 1u)) return;
    hipEvent_t e = take_event();
    SIC_HIP(hipEventRecord(e, s));
    g.open[kind] = e;
}

int64_t prof_end(int kind, hipStream_t s, double bytes, double flops) {
    if (!g.enabled || !g.open[kind]) return -1;
    hipEvent_t e = take_event();
    SIC_HIP(hipEventRecord(e, s));
    g.pending.push_back(Pending{kind, g.open[kind], e, bytes, flops});
    g.open[kind] = nullptr;
    return (int64_t)g.pending.size() - 1;
}

void prof_discard(int64_t handle) {
    if (handle >= 0 && handle < (int64_t)g.pending.size()) g.pending[handle].kind = -1;
}

void prof_scale(int64_t handle, double f) {
    if (handle >= 0 && handle < (int64_t)g.pending.size()) {
        g.pending[handle].bytes *= f;
        g.pending[handle].flops *= f;
    }
}

void prof_flush() {
    if (g.enabled && g.pending.size() >= 1024) resolve();
}

KernelStat prof_read(int kind) {
    resolve();
    return (kind >= 0 && kind < KK_COUNT) ? g.stat[kind] : KernelStat{};
}

}  // namespace sic

extern "C" {

void sic_profile_enable(int on) {
    try {
        sic::prof_enable(on != 0);
    } catch (...) {
    }
}

void sic_profile_select(uint32_t mask) { sic::g.mask = mask; }

void sic_profile_reset(void) {
    try {
        sic::prof_reset();
    } catch (...) {
    }
}

int sic_profile_read(int kind, int64_t* launches, double* milliseconds, double* bytes,
                     double* flops) {
    if (kind < 0 || kind >= sic::KK_COUNT) return -1;
    sic::KernelStat s;
    try {
        s = sic::prof_read(kind);
    } catch (...) {
        return -6;
    }
    if (launches) *launches = s.launches;
    if (milliseconds) *milliseconds = s.ms;
    if (bytes) *bytes = s.bytes;
    if (flops) *flops = s.flops;
    return 0;
}

const char* sic_profile_kernel_name(int kind) { return sic::kernel_kind_name(kind); }

}  // extern "C"
