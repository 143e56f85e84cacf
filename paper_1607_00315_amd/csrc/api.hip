// C-ABI entry points (sic.h, sic_steps.h): argument checks, error mapping,
// and thin wrappers over the solver and its steps.
#include <cmath>
#include <cstring>
#include <memory>
#include <new>

#include "sic_steps.h"
#include "solver.h"

struct sic_ctx {
    sic::Context c;
    // the last solve's problem storage (X and its copies, the CSR pair), reused
    // by the next solve on this context instead of allocated and freed per call
    std::unique_ptr<sic::Problem> P;
};

struct sic_prob {
    sic_ctx* ctx;
    sic::Problem P;
};

namespace {

thread_local std::string g_last_error;

template <class F>
int guard(F&& f) {
    try {
        return f();
    } catch (const sic::SicError& e) {
        g_last_error = e.what();
        return e.code;
    } catch (const sic::HipError& e) {
        g_last_error = e.what();
        return SIC_EHIP;
    } catch (const std::bad_alloc&) {
        g_last_error = "host allocation failed";
        return SIC_ENOMEM;
    } catch (const std::exception& e) {
        g_last_error = e.what();
        return SIC_EINTERNAL;
    }
}

void opts_from(sic::Context& C, const sic_options& o) {
    sic::Options& t = C.opt;
    t.block = o.block > 0 ? o.block : 256;
    t.cg_tol_I = o.cg_tol_I > 0 ? o.cg_tol_I : 1e-5;
    t.cg_tol_N = o.cg_tol_N > 0 ? o.cg_tol_N : 1e-4;
    t.cg_max_iter = o.cg_max_iter > 0 ? o.cg_max_iter : 1000;
    t.cd_tol = o.cd_tol > 0 ? o.cd_tol : 1e-4;
    t.cd_max_sweeps = o.cd_max_sweeps > 0 ? o.cd_max_sweeps : 20;
    t.cd_hessian_max = o.cd_hessian_max == 0 ? 4096 : (o.cd_hessian_max < 0 ? 0 : o.cd_hessian_max);
    t.pcd_min_coords = o.pcd_min_coords == 0 ? 4097 : (o.pcd_min_coords < 0 ? 0 : o.pcd_min_coords);
    t.ls_max_trials = o.ls_max_trials > 0 ? o.ls_max_trials : 31;
    t.max_cycles = o.max_cycles > 0 ? o.max_cycles : 100;
    t.flags = o.flags;
    t.precision = o.precision;
    C.trace = o.trace;
    C.trace_cap = o.trace ? o.trace_cap : 0;
    C.budget = o.hbm_budget;
    C.acct->budget = o.hbm_budget;
}

void check_block(int b) {
    if (b < 1 || b > 256) throw sic::SicError(SIC_EINVAL, "block size must lie in [1, 256]");
}

// scratch for the standalone CD / line-search steps
struct StepBufs {
    sic::DevBuf<double> wjj, S, A, delta;
    sic::DevBuf<int64_t> cptr;
    sic::DevBuf<int32_t> cp;
};

}  // namespace

namespace sic {

void context_init(Context& C, const sic_options& o) {
    check_block(o.block > 0 ? o.block : 256);
    C.device = o.device;
    SIC_HIP(hipSetDevice(o.device));
    int lds = 0;
    SIC_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, o.device));
    CD_MAX_LDS_BYTES = lds > 4096 ? (size_t)lds - 2048 : 0;
    if (o.stream) {
        C.stream = (hipStream_t)o.stream;
        C.own_stream = false;
    } else {
        SIC_HIP(hipStreamCreateWithFlags(&C.stream, hipStreamNonBlocking));
        C.own_stream = true;
    }
    SIC_HIP(hipStreamCreateWithFlags(&C.side, hipStreamNonBlocking));
    SIC_HIP(hipEventCreateWithFlags(&C.ev_fork, hipEventDisableTiming));
    SIC_HIP(hipEventCreateWithFlags(&C.ev_join, hipEventDisableTiming));
    SIC_HIP(hipHostMalloc((void**)&C.h_i64, 64 * sizeof(int64_t), hipHostMallocDefault));
    SIC_HIP(hipHostMalloc((void**)&C.h_f64, 64 * sizeof(double), hipHostMallocDefault));
    opts_from(C, o);
}

void context_release(Context& C) {
    (void)hipSetDevice(C.device);
    if (C.stream) (void)hipStreamSynchronize(C.stream);
    if (C.side) (void)hipStreamSynchronize(C.side);
    if (C.own_stream && C.stream) (void)hipStreamDestroy(C.stream);
    if (C.side) (void)hipStreamDestroy(C.side);
    if (C.ev_fork) (void)hipEventDestroy(C.ev_fork);
    if (C.ev_join) (void)hipEventDestroy(C.ev_join);
    C.side = nullptr;
    C.ev_fork = nullptr;
    C.ev_join = nullptr;
    if (C.h_i64) (void)hipHostFree(C.h_i64);
    if (C.h_f64) (void)hipHostFree(C.h_f64);
    C.stream = nullptr;
    C.h_i64 = nullptr;
    C.h_f64 = nullptr;
}

}  // namespace sic

namespace sic {
// implemented in solver.hip through these two helpers
struct LsPrepared;
}  // namespace sic

extern "C" {

void sic_options_default(sic_options* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->device = 0;
    o->precision = SIC_FP64;
    o->block = 256;
    o->cg_tol_I = 1e-5;
    o->cg_tol_N = 1e-4;
    o->cg_max_iter = 1000;
    o->cd_tol = 1e-4;
    o->cd_max_sweeps = 20;
    o->cd_hessian_max = 4096;
    o->pcd_min_coords = 4097;
    o->ls_max_trials = 31;
    o->max_cycles = 100;
}

const char* sic_strerror(int code) {
    switch (code) {
        case SIC_OK: return "ok";
        case SIC_EINVAL: return "invalid argument";
        case SIC_ENONFINITE: return "non-finite input";
        case SIC_ENOTPD: return "not positive definite";
        case SIC_ENOMEM: return "out of device memory or over the HBM budget";
        case SIC_ENOCONV: return "not converged within max_cycles";
        case SIC_EHIP: return "HIP runtime error";
        case SIC_ECANCELED: return "cancelled";
        case SIC_ETOOBIG: return "working set exceeds a kernel limit";
        case SIC_EINTERNAL: return "internal error";
        default: return "unknown error";
    }
}

const char* sic_last_error(void) { return g_last_error.c_str(); }

int sic_create(sic_ctx** out, const sic_options* opt) {
    if (!out) return SIC_EINVAL;
    *out = nullptr;
    return guard([&]() {
        sic_options o;
        sic_options_default(&o);
        if (opt) o = *opt;
        auto ctx = std::make_unique<sic_ctx>();
        sic::context_init(ctx->c, o);
        *out = ctx.release();
        return SIC_OK;
    });
}

void sic_destroy(sic_ctx* ctx) {
    if (!ctx) return;
    sic::context_release(ctx->c);
    delete ctx;
}

void sic_csr_free(sic_csr* a) {
    if (!a) return;
    free(a->rowptr);
    free(a->col);
    free(a->val);
    std::memset(a, 0, sizeof(*a));
}

int sic_solve(sic_ctx* ctx, const double* X, int64_t n, int64_t m, double lambda, double tol,
              sic_csr* A_out, sic_info* info) {
    if (!ctx || !X || !A_out || n < 1 || m < 1 || !(lambda >= 0.0) || !(tol > 0.0) ||
        !std::isfinite(lambda))
        return SIC_EINVAL;
    if (lambda == 0.0 && m <= n) {
        g_last_error = "lambda = 0 needs m > n (the sample covariance is singular otherwise)";
        return SIC_EINVAL;
    }
    return guard([&]() {
        sic::Context& C = ctx->c;
        sic::AccountScope scope(C.acct);
        SIC_HIP(hipSetDevice(C.device));
        if (!ctx->P) ctx->P = std::make_unique<sic::Problem>();
        sic::Problem& P = *ctx->P;
        try {
            sic::problem_init(C, P, X, SIC_X_F64, n, m, lambda);
            const int st = sic::solve_problem(C, P, tol, info);
            sic::get_A_host(C, P, A_out);
            return st;
        } catch (...) {
            ctx->P.reset();   // a failed solve keeps no problem storage
            throw;
        }
    });
}

int sic_solve_batch(sic_ctx* ctx, int count, const sic_problem* probs, sic_csr* A_out,
                    sic_info* info) {
    if (!ctx || count < 0 || (count > 0 && (!probs || !A_out))) return SIC_EINVAL;
    int first_bad = SIC_OK;
    int slot = 0;
    for (int k = 0; k < count; ++k) {
        const sic_problem& q = probs[k];
        const int nl = sic::request_results(q);
        sic_info* inf = info ? info + slot : nullptr;
        if (inf) std::memset(inf, 0, sizeof(sic_info) * nl);
        for (int l = 0; l < nl; ++l) std::memset(&A_out[slot + l], 0, sizeof(sic_csr));
        int st = guard([&]() {
            sic::Context& C = ctx->c;
            sic::AccountScope scope(C.acct);
            SIC_HIP(hipSetDevice(C.device));
            if (!ctx->P) ctx->P = std::make_unique<sic::Problem>();
            try {
                return sic::solve_request(C, *ctx->P, q, A_out + slot, inf);
            } catch (...) {
                ctx->P.reset();
                throw;
            }
        });
        if (st != SIC_OK && inf)
            for (int l = 0; l < nl; ++l)
                if (inf[l].status == SIC_OK) inf[l].status = st;
        if (st != SIC_OK && first_bad == SIC_OK) first_bad = st;
        slot += nl;
    }
    return first_bad;
}

// ------------------------------------------------------------------ steps

int sic_prob_create(sic_ctx* ctx, const double* X, int64_t n, int64_t m, double lambda,
                    sic_prob** out) {
    if (!ctx || !X || !out || n < 1 || m < 1 || !(lambda >= 0.0)) return SIC_EINVAL;
    *out = nullptr;
    return guard([&]() {
        sic::Context& C = ctx->c;
        sic::AccountScope scope(C.acct);
        SIC_HIP(hipSetDevice(C.device));
        auto p = std::make_unique<sic_prob>();
        p->ctx = ctx;
        sic::problem_init(C, p->P, X, SIC_X_F64, n, m, lambda, false);
        *out = p.release();
        return SIC_OK;
    });
}

void sic_prob_destroy(sic_prob* p) {
    // Device buffers are released with hipFree, which waits for pending work;
    // the owning context is not touched (it may already be destroyed).
    delete p;
}

int sic_prob_set_A(sic_prob* p, const sic_csr* A, double objective) {
    if (!p || !A) return SIC_EINVAL;
    return guard([&]() {
        sic::AccountScope scope(p->ctx->c.acct);
        sic::set_A_host(p->ctx->c, p->P, A);
        p->P.F = objective;
        return SIC_OK;
    });
}

int sic_prob_get_A(sic_prob* p, sic_csr* out) {
    if (!p || !out) return SIC_EINVAL;
    return guard([&]() {
        sic::AccountScope scope(p->ctx->c.acct);
        sic::get_A_host(p->ctx->c, p->P, out);
        return SIC_OK;
    });
}

double sic_prob_objective(sic_prob* p) { return p ? p->P.F : NAN; }

int sic_step_cov_block(sic_prob* p, int64_t j0, int b, double* out) {
    if (!p || !out || j0 < 0 || b < 1 || j0 + b > p->P.n) return SIC_EINVAL;
    return guard([&]() {
        sic::Context& C = p->ctx->c;
        sic::AccountScope scope(C.acct);
        C.work.SJ.reserve((size_t)p->P.n * b);
        sic::launch_sj_gemm_f64(p->P.X.p, p->P.n, p->P.m, j0, b, C.work.SJ.p, C.stream);
        SIC_HIP(hipMemcpyAsync(out, C.work.SJ.p, sizeof(double) * p->P.n * b,
                               hipMemcpyDeviceToHost, C.stream));
        SIC_HIP(hipStreamSynchronize(C.stream));
        return SIC_OK;
    });
}

int sic_step_cov_block_low(sic_prob* p, int64_t j0, int b, int x_dtype, double* out) {
    if (!p || !out || j0 < 0 || b < 1 || j0 + b > p->P.n ||
        (x_dtype != SIC_X_F32 && x_dtype != SIC_X_BF16))
        return SIC_EINVAL;
    return guard([&]() {
        sic::Context& C = p->ctx->c;
        sic::AccountScope scope(C.acct);
        const size_t count = (size_t)p->P.n * p->P.m;
        sic::DevBuf<float> xf;
        sic::DevBuf<uint16_t> xb;
        if (x_dtype == SIC_X_F32) xf.reserve(count); else xb.reserve(count);
        sic::launch_narrow(p->P.X.p, (int64_t)count, x_dtype == SIC_X_F32 ? xf.p : nullptr,
                           x_dtype == SIC_X_BF16 ? xb.p : nullptr, C.stream);
        C.work.SJ.reserve((size_t)p->P.n * b);
        sic::launch_sj_gemm_low(x_dtype == SIC_X_BF16 ? (const void*)xb.p : (const void*)xf.p,
                                x_dtype == SIC_X_BF16, p->P.n, p->P.m, j0, b, C.work.SJ.p,
                                C.stream);
        SIC_HIP(hipMemcpyAsync(out, C.work.SJ.p, sizeof(double) * p->P.n * b,
                               hipMemcpyDeviceToHost, C.stream));
        SIC_HIP(hipStreamSynchronize(C.stream));
        return SIC_OK;
    });
}

int sic_step_cov_pairs(sic_prob* p, const int32_t* rows, const int32_t* cols, int64_t count,
                       double* out) {
    if (!p || count < 0 || (count > 0 && (!rows || !cols || !out))) return SIC_EINVAL;
    for (int64_t t = 0; t < count; ++t)
        if (rows[t] < 0 || rows[t] >= p->P.n || cols[t] < 0 || cols[t] >= p->P.n) return SIC_EINVAL;
    if (count == 0) return SIC_OK;
    return guard([&]() {
        sic::Context& C = p->ctx->c;
        sic::AccountScope scope(C.acct);
        sic::DevBuf<int32_t> r, c;
        sic::DevBuf<double> o;
        r.reserve(count); c.reserve(count); o.reserve(count);
        SIC_HIP(hipMemcpyAsync(r.p, rows, sizeof(int32_t) * count, hipMemcpyHostToDevice, C.stream));
        SIC_HIP(hipMemcpyAsync(c.p, cols, sizeof(int32_t) * count, hipMemcpyHostToDevice, C.stream));
        sic::launch_sddmm(p->P.Xt.p, p->P.m, r.p, c.p, count, o.p, C.stream);
        SIC_HIP(hipMemcpyAsync(out, o.p, sizeof(double) * count, hipMemcpyDeviceToHost, C.stream));
        SIC_HIP(hipStreamSynchronize(C.stream));
        return SIC_OK;
    });
}

int sic_step_inverse_columns(sic_prob* p, const int32_t* cols, int k, double tol, int max_iter,
                             double* out, int* iterations, double* max_rel_residual) {
    if (!p || !cols || !out || k < 1 || !(tol > 0.0) || max_iter < 1) return SIC_EINVAL;
    for (int j = 0; j < k; ++j)
        if (cols[j] < 0 || cols[j] >= p->P.n) return SIC_EINVAL;
    return guard([&]() {
        sic::Context& C = p->ctx->c;
        sic::AccountScope scope(C.acct);
        const int64_t n = p->P.n;
        sic::DevBuf<int32_t> dc;
        sic::DevBuf<double> W;
        dc.reserve(k);
        W.reserve((size_t)n * k);
        SIC_HIP(hipMemcpyAsync(dc.p, cols, sizeof(int32_t) * k, hipMemcpyHostToDevice, C.stream));
        sic::CGResult r = sic::block_cg(p->P.Acur(), dc.p, k, W.p, k, tol, max_iter, C.work.cg, C.stream);
        SIC_HIP(hipMemcpyAsync(out, W.p, sizeof(double) * n * k, hipMemcpyDeviceToHost, C.stream));
        SIC_HIP(hipStreamSynchronize(C.stream));
        if (iterations) *iterations = r.iterations;
        if (max_rel_residual) *max_rel_residual = r.max_rel_res;
        return SIC_OK;
    });
}

int sic_step_inverse_columns_noalloc(const int64_t* rowptr, const int32_t* col,
                                     const double* val, int64_t n, int64_t nnz,
                                     const int32_t* cols, int k, double tol, int max_iter,
                                     double* W, void* stream, int* iterations,
                                     double* max_rel_residual) {
    if (!rowptr || !col || !val || !cols || !W || n < 1 || nnz < n || k < 1 || !(tol > 0.0) ||
        max_iter < 1)
        return SIC_EINVAL;
    return guard([&]() {
        const sic::CGResult r =
            sic::block_cg_noalloc(rowptr, col, val, n, nnz, cols, k, W, tol, max_iter,
                                  static_cast<hipStream_t>(stream));
        if (iterations) *iterations = r.iterations;
        if (max_rel_residual) *max_rel_residual = r.max_rel_res;
        return SIC_OK;
    });
}

size_t sic_step_inverse_columns_noalloc_limit(int64_t n, int64_t nnz, int k) {
    if (n < 1 || nnz < 0 || k < 1 || k > sic::cg_noalloc_max_k()) return 0;
    const size_t need = sic::cg_noalloc_bytes(n, nnz, k);
    return need <= sic::cg_noalloc_capacity() ? need : 0;
}

int sic_step_set_level(sic_prob* p, const int64_t* keys, int64_t count) {
    if (!p || count < 0 || (count > 0 && !keys)) return SIC_EINVAL;
    return guard([&]() {
        sic::AccountScope scope(p->ctx->c.acct);
        sic::set_level_keys(p->ctx->c, p->P, keys, count);
        return SIC_OK;
    });
}

static void fill_block_result(const sic::BlockResult& R, sic_block_result* res) {
    if (!res) return;
    res->E = R.E;
    res->n_neighbors = R.nN;
    res->n_level_nbrs = R.nC;
    res->n_coords = R.ncoord;
    res->cg_iterations_I = R.cg_iters_I;
    res->cg_iterations_N = R.cg_iters_N;
    res->cd_sweeps = R.cd_sweeps;
    res->cd_last_max_mu = R.cd_last_maxmu;
    res->alpha = R.alpha;
    res->dF = R.dF;
    res->trials = R.trials;
    res->nnz_after = R.nnz_after;
}

int sic_step_block(sic_prob* p, int64_t j0, int b, int level, double tol_I, double tol_N,
                   sic_block_result* res) {
    if (!p || j0 < 0 || b < 1 || b > 256 || j0 + b > p->P.n || level < 0) return SIC_EINVAL;
    return guard([&]() {
        sic::Context& C = p->ctx->c;
        sic::AccountScope scope(C.acct);
        const double tI = tol_I > 0 ? tol_I : C.opt.cg_tol_I;
        const double tN = tol_N > 0 ? tol_N : C.opt.cg_tol_N;
        sic::BlockResult R = sic::block_update(C, p->P, j0, b, level == 0, false, tI, tN);
        fill_block_result(R, res);
        return SIC_OK;
    });
}

int sic_step_last_block(sic_prob* p, int64_t* colptr, int32_t* rows, double* g, int32_t* nbrs,
                        int32_t* coord_rows, int32_t* coord_cols, double* delta, double* wjj) {
    if (!p) return SIC_EINVAL;
    return guard([&]() {
        sic::Context& C = p->ctx->c;
        sic::AccountScope scope(C.acct);
        sic::BlockWork& W = C.work;
        const sic::BlockResult& R = C.last;
        hipStream_t s = C.stream;
        const int b = R.b;
        if (colptr) SIC_HIP(hipMemcpyAsync(colptr, W.colptr.p, sizeof(int64_t) * (b + 1), hipMemcpyDeviceToHost, s));
        if (rows && R.E) SIC_HIP(hipMemcpyAsync(rows, W.e_row.p, sizeof(int32_t) * R.E, hipMemcpyDeviceToHost, s));
        if (g && R.E) SIC_HIP(hipMemcpyAsync(g, W.e_g.p, sizeof(double) * R.E, hipMemcpyDeviceToHost, s));
        std::vector<int32_t> Jp(R.jp);
        SIC_HIP(hipMemcpyAsync(Jp.data(), W.Jp.p, sizeof(int32_t) * R.jp, hipMemcpyDeviceToHost, s));
        std::vector<int32_t> cp(std::max<int64_t>(R.ncoord, 1)), cc(std::max<int64_t>(R.ncoord, 1));
        if (R.ncoord) {
            SIC_HIP(hipMemcpyAsync(cp.data(), W.c_p.p, sizeof(int32_t) * R.ncoord, hipMemcpyDeviceToHost, s));
            SIC_HIP(hipMemcpyAsync(cc.data(), W.c_ci.p, sizeof(int32_t) * R.ncoord, hipMemcpyDeviceToHost, s));
        }
        if (delta && R.ncoord) SIC_HIP(hipMemcpyAsync(delta, W.delta.p, sizeof(double) * R.ncoord, hipMemcpyDeviceToHost, s));
        if (wjj) SIC_HIP(hipMemcpyAsync(wjj, W.WJJ.p, sizeof(double) * R.jp * R.jp, hipMemcpyDeviceToHost, s));
        SIC_HIP(hipStreamSynchronize(s));
        if (nbrs)
            for (int64_t t = 0; t < R.nN; ++t) nbrs[t] = Jp[b + t];
        for (int64_t t = 0; t < R.ncoord; ++t) {
            if (coord_rows) coord_rows[t] = Jp[cp[t]];
            if (coord_cols) coord_cols[t] = (int32_t)(R.j0 + cc[t]);
        }
        return SIC_OK;
    });
}

int sic_step_sweep(sic_prob* p, int level, double tol_I, double tol_N, double* kkt_max,
                   double* kkt_l1) {
    if (!p || level < 0) return SIC_EINVAL;
    return guard([&]() {
        sic::Context& C = p->ctx->c;
        sic::AccountScope scope(C.acct);
        const double tI = tol_I > 0 ? tol_I : C.opt.cg_tol_I;
        const double tN = tol_N > 0 ? tol_N : C.opt.cg_tol_N;
        sic::SweepResult S = sic::sweep(C, p->P, level == 0, tI, tN);
        if (kkt_max) *kkt_max = S.kkt_max;
        if (kkt_l1) *kkt_l1 = S.kkt_l1;
        return SIC_OK;
    });
}

int sic_step_kkt(sic_prob* p, double tol_cg, double* kkt_max, double* kkt_l1) {
    if (!p || !(tol_cg > 0.0)) return SIC_EINVAL;
    return guard([&]() {
        sic::AccountScope scope(p->ctx->c.acct);
        double l1 = 0.0;
        const double m = sic::exact_kkt(p->ctx->c, p->P, tol_cg, &l1);
        if (kkt_max) *kkt_max = m;
        if (kkt_l1) *kkt_l1 = l1;
        return SIC_OK;
    });
}

}  // extern "C"

namespace sic {
// standalone steps (d) and (e) on caller data
int step_cd_impl(Context& C, int jp, int b, const double* wjj, const int64_t* cptr,
                 const int32_t* cp, const double* S, const double* A, double lambda, int max_sweeps,
                 double tol, double* delta_out, double* stats_out);
int step_ls_impl(Context& C, int jp, int b, const double* wjj, const int64_t* cptr,
                 const int32_t* cp, const double* S, const double* A, const double* delta,
                 double lambda, double* alpha, double* dF, int* trials, double* logdet_out,
                 int n_alpha);
}  // namespace sic

extern "C" {

int sic_step_cd(sic_ctx* ctx, int jp, int b, const double* wjj, const int64_t* cptr,
                const int32_t* cp, const double* S, const double* A, double lambda,
                int max_sweeps, double tol, double* delta_out, double* stats_out) {
    if (!ctx || !wjj || !cptr || b < 1 || b > 256 || jp < b || max_sweeps < 1 || !delta_out)
        return SIC_EINVAL;
    const int64_t nc = cptr[b];
    if (cptr[0] != 0 || nc < 0) return SIC_EINVAL;
    for (int i = 0; i < b; ++i)
        if (cptr[i + 1] < cptr[i]) return SIC_EINVAL;
    for (int64_t t = 0; t < nc; ++t)
        if (cp[t] < 0 || cp[t] >= jp) return SIC_EINVAL;
    return guard([&]() {
        sic::AccountScope scope(ctx->c.acct);
        return sic::step_cd_impl(ctx->c, jp, b, wjj, cptr, cp, S, A, lambda, max_sweeps, tol,
                                 delta_out, stats_out);
    });
}

int sic_step_linesearch(sic_ctx* ctx, int jp, int b, const double* wjj, const int64_t* cptr,
                        const int32_t* cp, const double* S, const double* A, const double* delta,
                        double lambda, double* alpha, double* dF, int* trials,
                        double* logdet_out, int n_alpha) {
    if (!ctx || !wjj || !cptr || !delta || b < 1 || b > 256 || jp < b) return SIC_EINVAL;
    const int64_t nc = cptr[b];
    if (cptr[0] != 0 || nc < 0) return SIC_EINVAL;
    for (int i = 0; i < b; ++i)
        if (cptr[i + 1] < cptr[i]) return SIC_EINVAL;
    for (int64_t t = 0; t < nc; ++t)
        if (cp[t] < 0 || cp[t] >= jp) return SIC_EINVAL;
    return guard([&]() {
        sic::AccountScope scope(ctx->c.acct);
        return sic::step_ls_impl(ctx->c, jp, b, wjj, cptr, cp, S, A, delta, lambda, alpha, dF,
                                 trials, logdet_out, n_alpha);
    });
}

int sic_hierarchy(int64_t n, const int64_t* supp_keys, int64_t n_supp, const int64_t* free_keys,
                  const double* free_absg, int64_t n_free, int64_t* ranking_out,
                  int64_t* ranking_len, int64_t* sizes_out, int* n_levels) {
    if (n < 1 || n_supp < 0 || n_free < 0 || (n_supp && !supp_keys) ||
        (n_free && (!free_keys || !free_absg)) || !ranking_out || !sizes_out || !n_levels)
        return SIC_EINVAL;
    return guard([&]() {
        std::vector<int64_t> supp(supp_keys, supp_keys + n_supp);
        std::vector<int64_t> fk(free_keys, free_keys + n_free);
        std::vector<double> fg(free_absg, free_absg + n_free);
        std::vector<int64_t> ranking, sizes;
        sic::hierarchy_host(n, supp, fk, fg, ranking, sizes);
        if ((int64_t)ranking.size() > n_supp + n_free || sizes.size() > 64)
            throw sic::SicError(SIC_EINTERNAL, "hierarchy output larger than its buffers");
        std::copy(ranking.begin(), ranking.end(), ranking_out);
        if (ranking_len) *ranking_len = (int64_t)ranking.size();
        std::copy(sizes.begin(), sizes.end(), sizes_out);
        *n_levels = (int)sizes.size();
        return SIC_OK;
    });
}

}  // extern "C"
