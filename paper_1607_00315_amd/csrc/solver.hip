// The multilevel block coordinate-descent solver on the host side:
//   block_update  one block of Algorithm 2 at the finest level or, restricted
//                 to a level set C_l, at a coarse level (Section 7, App. A.2)
//   sweep         one relaxation = the blocks in order
//   solve_problem Algorithm 1 cycles until the KKT target
// Every arithmetic step runs in the kernels of this library; the host only
// sequences launches, reads back the few sizes that shape the next launch,
// and builds the nested level sets from the recorded free set.
#include <algorithm>
#include <chrono>
#include <functional>
#include <cmath>
#include <cstring>
#include <new>
#include <numeric>

#include "profiler.h"
#include "solver.h"

namespace sic {

// line-search trials per launch
constexpr int LS_BATCH = 8;

size_t CD_MAX_LDS_BYTES = 65536;

namespace {
std::shared_ptr<MemAccount>& default_account() {
    static std::shared_ptr<MemAccount> a = std::make_shared<MemAccount>();
    return a;
}
thread_local std::shared_ptr<MemAccount> t_account;
}  // namespace

const std::shared_ptr<MemAccount>& current_account() {
    return t_account ? t_account : default_account();
}

AccountScope::AccountScope(const std::shared_ptr<MemAccount>& a) : prev_(t_account) {
    t_account = a;
}
AccountScope::~AccountScope() { t_account = prev_; }

namespace {
thread_local bool t_blocking_waits = false;
}  // namespace

void set_blocking_waits(bool on) { t_blocking_waits = on; }

void stream_wait(hipStream_t s) {
    // one event per host thread and device (serving threads wait concurrently)
    thread_local std::vector<std::pair<int, hipEvent_t>> events;
    int dev = 0;
    SIC_HIP(hipGetDevice(&dev));
    hipEvent_t ev = nullptr;
    for (auto& e : events)
        if (e.first == dev) ev = e.second;
    if (!ev) {
        SIC_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        events.emplace_back(dev, ev);
    }
    SIC_HIP(hipEventRecord(ev, s));
    if (t_blocking_waits) {
        SIC_HIP(hipEventSynchronize(ev));
        return;
    }
    const auto t0 = std::chrono::steady_clock::now();
    for (;;) {
        const hipError_t e = hipEventQuery(ev);
        if (e == hipSuccess) return;
        if (e != hipErrorNotReady) SIC_HIP(e);
        if (std::chrono::steady_clock::now() - t0 > std::chrono::microseconds(2000)) break;
    }
    SIC_HIP(hipEventSynchronize(ev));
}

namespace {

constexpr int ROWS_PER_TILE = 32;

void sync(Context& C) { stream_wait(C.stream); }

int64_t read_i64(Context& C, const int64_t* d) {
    SIC_HIP(hipMemcpyAsync(C.h_i64, d, sizeof(int64_t), hipMemcpyDeviceToHost, C.stream));
    sync(C);
    return C.h_i64[0];
}

// The screening's free pairs (rows, gradients, S, A, W entries): at most one
// per entry of the n x b block, so the emit pass runs without the count.
void reserve_free_lists(BlockWork& W, size_t nb) {
    W.e_row.reserve(nb); W.e_g.reserve(nb); W.e_s.reserve(nb); W.e_a.reserve(nb); W.e_w.reserve(nb);
}

void ensure_flags(Context& C, int64_t n, int b) {
    BlockWork& W = C.work;
    if (W.n_init == n && W.b_init >= b) return;
    W.nflag.reserve(n);
    W.cflag.reserve(n);
    W.lmap.reserve(n);
    W.cmap.reserve(n);
    SIC_HIP(hipMemsetAsync(W.nflag.p, 0, sizeof(int32_t) * n, C.stream));
    SIC_HIP(hipMemsetAsync(W.cflag.p, 0, sizeof(int32_t) * n, C.stream));
    launch_fill_i32(W.lmap.p, n, -1, C.stream);
    launch_fill_i32(W.cmap.p, n, -1, C.stream);
    W.ANEW.reserve((size_t)n * b);
    SIC_HIP(hipMemsetAsync(W.ANEW.p, 0, sizeof(double) * n * b, C.stream));
    W.n_init = n;
    W.b_init = b;
}

// The line search's outputs, written by its kernels straight into pinned
// staging: W_II's log det and PD flag, two per trial, then the trials' linear
// terms (2 + 3 LS_BATCH doubles).
double* ls_out(Context& C) { return C.h_f64; }

struct LineSearch {
    double alpha = 0, dF = 0;
    int trials = 0;
    bool wii_pd = true;
};

// Every buffer of the line search, sized before any of its work is queued.
void ls_reserve(Context& C, int b, int64_t nN) {
    BlockWork& W = C.work;
    const size_t bb = (size_t)b * b;
    W.Dinv.reserve(8 * 1024);
    W.Rb.reserve(bb); W.D11.reserve(bb); W.Mo.reserve(bb); W.Pm.reserve(bb);
    W.T1.reserve(bb); W.T2.reserve(bb); W.D1.reserve(bb); W.X.reserve(bb); W.XtX.reserve(bb);
    W.RPR.reserve(bb); W.E1.reserve(bb); W.E2.reserve(bb);
    W.Y.reserve((size_t)std::max<int64_t>(nN, 1) * b);
    W.C.reserve(LS_BATCH * bb);
}

// R R^T = W_II (R lower, in W.Rb; its diagonal-block inverses in W.Dinv), on stream st.
void ls_factor_wii(Context& C, int jp, int b, hipStream_t st) {
    BlockWork& W = C.work;
    launch_copy_block(W.WJJ.p, jp, b, W.Rb.p, st);
    launch_chol(W.Rb.p, (int64_t)b * b, 1, b, b, 0, ls_out(C), st, W.Dinv.p);
    launch_zero_upper(W.Rb.p, b, b, st);
}

// Whitened Schur-complement matrices E1, E2 of the line search (see k_dense.hip):
// log det(A + a Delta) - log det A = log det(I + a E1 + a^2 E2).
// factored: W_II's factor was queued on the side stream (the main stream
// waits for it here); otherwise it is computed in order.
void ls_prepare(Context& C, int jp, int b, int64_t nN, bool factored) {
    BlockWork& W = C.work;
    hipStream_t s = C.stream;
    // the side stream may still be factoring W_II into Rb / Dinv: those were
    // sized before the fork, and sizing them again must not move them
    const void* held[2] = {W.Rb.p, W.Dinv.p};
    ls_reserve(C, b, nN);
    if (factored && (held[0] != W.Rb.p || held[1] != W.Dinv.p))
        throw SicError(SIC_EINTERNAL, "a buffer of the side stream moved before its join");
    if (factored)
        SIC_HIP(hipStreamWaitEvent(s, C.ev_join, 0));
    else
        ls_factor_wii(C, jp, b, s);
    launch_ls_terms(W.cptr.p, W.c_p.p, W.delta.p, W.WJJ.p, jp, b, (int)nN, W.D11.p, W.Mo.p, W.Y.p,
                    W.Pm.p, s);
    // D1 = R^T Delta_II R and RPR = R^T P R on the side stream, beside the K1
    // chain on the main one
    hipStream_t side = C.side;
    SIC_HIP(hipEventRecord(C.ev_fork, s));
    SIC_HIP(hipStreamWaitEvent(side, C.ev_fork, 0));
    launch_gemm_small(b, b, b, 1.0, W.D11.p, b, 0, W.Rb.p, b, 0, 0.0, W.T1.p, b, side);
    launch_gemm_small(b, b, b, 1.0, W.Rb.p, b, 1, W.T1.p, b, 0, 0.0, W.D1.p, b, side);
    launch_gemm_small(b, b, b, 1.0, W.Pm.p, b, 0, W.Rb.p, b, 0, 0.0, W.T2.p, b, side);
    launch_gemm_small(b, b, b, 1.0, W.Rb.p, b, 1, W.T2.p, b, 0, 0.0, W.RPR.p, b, side);
    SIC_HIP(hipEventRecord(C.ev_join, side));
    // X = R^{-1} (M^T R) = K1^T, XtX = K1 K1^T
    launch_gemm_small(b, b, b, 1.0, W.Mo.p, b, 1, W.Rb.p, b, 0, 0.0, W.X.p, b, s);
    launch_trsm_lower(W.Rb.p, b, b, W.Dinv.p, W.X.p, b, b, 0, s);
    launch_gemm_small(b, b, b, 1.0, W.X.p, b, 1, W.X.p, b, 0, 0.0, W.XtX.p, b, s);
    SIC_HIP(hipStreamWaitEvent(s, C.ev_join, 0));
    launch_ls_e(W.D1.p, W.X.p, W.XtX.p, W.RPR.p, b, W.E1.p, W.E2.p, s);
}

// Evaluate the nt <= LS_BATCH trial steps alpha = 2^-(first + t): log det
// change, PD flag, linear terms, read back in one copy to pinned memory.
// Returns whether W_II itself factored (positive definite).
bool ls_eval(Context& C, int b, int64_t ncoord, double lam, int first, int nt,
             double* logdet, int* pd, double* lin) {
    BlockWork& W = C.work;
    hipStream_t s = C.stream;
    const size_t bb = (size_t)b * b;
    double* h_out = ls_out(C);
    double* dlin = h_out + 2 + 2 * LS_BATCH;
    launch_ls_trials(W.E1.p, W.E2.p, b, first, nt, W.C.p, s);
    launch_chol(W.C.p, (int64_t)bb, nt, b, b, 1, h_out + 2, s);
    launch_ls_linear(ncoord, W.c_p.p, W.c_ci.p, W.c_S.p, W.c_A.p, W.delta.p, lam, first, nt,
                     dlin, s);
    sync(C);
    for (int t = 0; t < nt; ++t) {
        logdet[t] = h_out[2 + 2 * t];
        pd[t] = h_out[2 + 2 * t + 1] != 0.0;
        lin[t] = h_out[2 + 2 * LS_BATCH + t];
    }
    return h_out[1] != 0.0;
}

// Step length by the backtracking rule of Section 6.1.2: alpha = 2^-i,
// non-PD trials skipped, then continue while F keeps decreasing; alpha = 0
// when no trial decreases F. Trials are evaluated LS_BATCH at a time (one
// workgroup each, so a batch costs one factorization's latency).
LineSearch line_search(Context& C, double lam, int jp, int b, int64_t nN, int64_t ncoord,
                       bool factored = false) {
    ls_prepare(C, jp, b, nN, factored);
    LineSearch res;
    bool have = false, stop = false;
    double best_a = 0.0, best_f = 0.0;
    int i = 0;
    const int max_trials = std::max(1, C.opt.ls_max_trials);
    while (!stop && i < max_trials) {
        const int nt = std::min(LS_BATCH, max_trials - i);
        double al[LS_BATCH], ld[LS_BATCH], lin[LS_BATCH];
        int pd[LS_BATCH];
        for (int t = 0; t < nt; ++t) al[t] = std::ldexp(1.0, -(i + t));
        res.wii_pd = ls_eval(C, b, ncoord, lam, i, nt, ld, pd, lin);
        if (!res.wii_pd) break;
        for (int t = 0; t < nt; ++t) {
            res.trials++;
            if (!pd[t]) {
                if (have) { stop = true; break; }
                continue;
            }
            const double f = lin[t] - ld[t];
            if (!have || f < best_f) {
                have = true;
                best_a = al[t];
                best_f = f;
                continue;
            }
            stop = true;
            break;
        }
        i += nt;
    }
    if (have && best_f < 0.0 && res.wii_pd) {
        res.alpha = best_a;
        res.dF = best_f;
    }
    return res;
}

}  // namespace

// ------------------------------------------------------------------ setup

__global__ void k_to_f64_from_f32(const float* __restrict__ in, int64_t count, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = (double)in[i];
}

__global__ void k_to_f64_from_bf16(const uint16_t* __restrict__ in, int64_t count, double* __restrict__ out) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) out[i] = (double)__uint_as_float(((unsigned int)in[i]) << 16);
}

void problem_init(Context& C, Problem& P, const void* X, int x_dtype, int64_t n, int64_t m,
                  double lam, bool warm_allowed) {
    hipStream_t s = C.stream;
    P.n = n;
    P.m = m;
    P.lam = lam;
    const size_t count = (size_t)n * m;
    P.X.reserve(count);
    hipPointerAttribute_t attr;
    bool on_device = false;
    if (hipPointerGetAttributes(&attr, X) == hipSuccess)
        on_device = attr.type == hipMemoryTypeDevice;
    (void)hipGetLastError();
    size_t esz = x_dtype == SIC_X_F64 ? 8 : (x_dtype == SIC_X_F32 ? 4 : 2);
    if (x_dtype == SIC_X_F64) {
        SIC_HIP(hipMemcpyAsync(P.X.p, X, count * esz,
                               on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
    } else {
        DevBuf<char>& tmp = C.work.xstage;   // kept: no free (and no device sync) per problem
        tmp.reserve(count * esz);
        SIC_HIP(hipMemcpyAsync(tmp.p, X, count * esz,
                               on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice, s));
        const unsigned grid = (unsigned)((count + 255) / 256);
        if (x_dtype == SIC_X_F32)
            hipLaunchKernelGGL(k_to_f64_from_f32, dim3(grid), dim3(256), 0, s,
                               (const float*)tmp.p, (int64_t)count, P.X.p);
        else
            hipLaunchKernelGGL(k_to_f64_from_bf16, dim3(grid), dim3(256), 0, s,
                               (const uint16_t*)tmp.p, (int64_t)count, P.X.p);
        SIC_CHECK_LAUNCH();
        sync(C);
    }
    P.narrow = C.opt.precision == SIC_MIXED;
    if (P.narrow) {
        P.Xf.reserve(count);
        P.Xb.reserve(count);
        launch_narrow(P.X.p, (int64_t)count, P.Xf.p, P.Xb.p, s);
    }
    P.Xt.reserve(count);
    launch_transpose(P.X.p, m, n, P.Xt.p, s);
    P.diagS.reserve(n);
    launch_diag_s(P.Xt.p, n, m, P.diagS.p, s);
    std::vector<double> d(n);
    SIC_HIP(hipMemcpyAsync(d.data(), P.diagS.p, sizeof(double) * n, hipMemcpyDeviceToHost, s));
    sync(C);
    for (double v : d)
        if (!std::isfinite(v)) throw SicError(SIC_ENONFINITE, "non-finite value in X");
    set_identity(C, P);
    double tr = 0.0;
    for (double v : d) tr += v;
    P.F = tr + lam * (double)n;   // F(I) = -log det I + tr(S) + lam * n
    P.level_set = false;
    P.perm.clear();
    P.scache = warm_allowed && !(C.opt.flags & SIC_FLAG_NO_S_CACHE) && warm_store_fits(n);
    P.s_cached.assign(P.scache ? (size_t)n : 0, 0);
    if (P.scache) P.Scache.reserve((size_t)n * n);
    P.warm = warm_allowed && !(C.opt.flags & SIC_FLAG_NO_WARM_CG) && warm_store_fits(n);
    if (P.warm) {
        P.Wst.reserve((size_t)n * n);
        P.Wvalid.reserve(n);
        SIC_HIP(hipMemsetAsync(P.Wvalid.p, 0, (size_t)n, s));
    }
}

void set_identity(Context& C, Problem& P) {
    const int64_t n = P.n;
    DevCSR& A = P.A[P.cur];
    std::vector<int64_t> rp(n + 1);
    std::vector<int32_t> cl(n);
    std::vector<double> vl(n, 1.0);
    for (int64_t i = 0; i <= n; ++i) rp[i] = i;
    for (int64_t i = 0; i < n; ++i) cl[i] = (int32_t)i;
    A.n = n;
    A.nnz = n;
    A.rowptr.reserve(n + 1);
    A.col.reserve(n);
    A.val.reserve(n);
    SIC_HIP(hipMemcpyAsync(A.rowptr.p, rp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, C.stream));
    SIC_HIP(hipMemcpyAsync(A.col.p, cl.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, C.stream));
    SIC_HIP(hipMemcpyAsync(A.val.p, vl.data(), sizeof(double) * n, hipMemcpyHostToDevice, C.stream));
    sync(C);
    P.max_nnz = n;
}

void set_A_host(Context& C, Problem& P, const sic_csr* in) {
    const int64_t n = P.n;
    if (!in || in->n != n || !in->rowptr || (in->nnz > 0 && (!in->col || !in->val)))
        throw SicError(SIC_EINVAL, "warm start CSR does not match the problem");
    if (in->rowptr[0] != 0 || in->rowptr[n] != in->nnz)
        throw SicError(SIC_EINVAL, "warm start CSR row pointers are inconsistent");
    bool diag_ok = true;
    for (int64_t i = 0; i < n && diag_ok; ++i) {
        bool found = false;
        for (int64_t e = in->rowptr[i]; e < in->rowptr[i + 1]; ++e) {
            if (!std::isfinite(in->val[e])) throw SicError(SIC_ENONFINITE, "non-finite warm start");
            if (e > in->rowptr[i] && in->col[e] <= in->col[e - 1])
                throw SicError(SIC_EINVAL, "warm start columns must be sorted and unique");
            if (in->col[e] == i) found = in->val[e] > 0.0;
        }
        diag_ok = found;
    }
    if (!diag_ok) throw SicError(SIC_ENOTPD, "warm start has a non-positive diagonal");
    DevCSR& A = P.A[P.cur];
    A.n = n;
    A.nnz = in->nnz;
    A.rowptr.reserve(n + 1);
    A.col.reserve(std::max<int64_t>(in->nnz, 1));
    A.val.reserve(std::max<int64_t>(in->nnz, 1));
    SIC_HIP(hipMemcpyAsync(A.rowptr.p, in->rowptr, sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, C.stream));
    if (in->nnz) {
        SIC_HIP(hipMemcpyAsync(A.col.p, in->col, sizeof(int32_t) * in->nnz, hipMemcpyHostToDevice, C.stream));
        SIC_HIP(hipMemcpyAsync(A.val.p, in->val, sizeof(double) * in->nnz, hipMemcpyHostToDevice, C.stream));
    }
    sync(C);
    P.max_nnz = std::max(P.max_nnz, in->nnz);
}

// Largest n for which a warm start is checked by a dense factorization
// (8 n^2 bytes of device scratch, 16 GiB here).
constexpr int64_t DENSE_CHECK_MAX_N = 46340;

// A warm start must be positive definite (the line search of Section 6.1.2
// starts from a PD iterate and keeps it PD). Up to DENSE_CHECK_MAX_N
// variables this is decided exactly: the iterate is expanded to a dense
// matrix and factored by a right-looking blocked Cholesky on the GPU (256 x
// 256 diagonal tiles by k_chol, the panel by the blocked triangular solve,
// the trailing update on the matrix cores), and F(A0) = -log det A0 +
// tr(S A0) + lambda ||A0||_1 (eq. (MLE_l1_prior)) follows from the pivots, the
// sampled entries S_ij on the pattern of A0 and the values. Above that size
// only strict diagonal dominance with a positive diagonal (a sufficient
// condition, Gershgorin) is accepted and F(A0) is not known (NaN).
// Returns F(A0); throws SIC_ENOTPD when A0 is not positive definite.
double warm_start_objective(Context& C, Problem& P, const sic_csr* in) {
    const int64_t n = P.n;
    hipStream_t s = C.stream;
    double l1 = 0.0;
    for (int64_t e = 0; e < in->nnz; ++e) l1 += std::fabs(in->val[e]);
    if (n > DENSE_CHECK_MAX_N) {
        for (int64_t i = 0; i < n; ++i) {
            double d = 0.0, off = 0.0;
            for (int64_t e = in->rowptr[i]; e < in->rowptr[i + 1]; ++e) {
                if (in->col[e] == i)
                    d = in->val[e];
                else
                    off += std::fabs(in->val[e]);
            }
            if (!(d > off))
                throw SicError(SIC_ENOTPD, "warm start above the dense-check size must be strictly "
                                           "diagonally dominant with a positive diagonal");
        }
        return NAN;
    }
    DevCSR& A = P.Acur();
    DevBuf<double> D;
    D.reserve((size_t)n * n);
    launch_csr_to_dense(A.rowptr.p, A.col.p, A.val.p, n, D.p, s);
    constexpr int T = 256;
    const int tiles = (int)((n + T - 1) / T);
    DevBuf<double> outs, dinv;
    outs.reserve(2 * (size_t)tiles);
    dinv.reserve(8 * 1024);
    for (int t = 0; t < tiles; ++t) {
        const int64_t k0 = (int64_t)t * T, k1 = std::min<int64_t>(k0 + T, n);
        const int nb = (int)(k1 - k0);
        double* Dkk = D.p + k0 * n + k0;
        launch_chol(Dkk, 0, 1, nb, (int)n, 0, outs.p + 2 * t, s, dinv.p);
        if (k1 < n) {
            const int rest = (int)(n - k1);
            double* X = D.p + k0 * n + k1;   // row panel: becomes L_kk^{-1} A_{k, k1:}
            launch_trsm_lower(Dkk, nb, (int)n, dinv.p, X, rest, (int)n, 0, s);
            launch_gemm_small(rest, rest, nb, -1.0, X, (int)n, 1, X, (int)n, 0, 1.0,
                              D.p + k1 * n + k1, (int)n, s);
        }
    }
    std::vector<double> o(2 * (size_t)tiles);
    SIC_HIP(hipMemcpyAsync(o.data(), outs.p, sizeof(double) * o.size(), hipMemcpyDeviceToHost, s));
    // tr(S A0) from the sampled entries on the pattern of A0
    std::vector<int32_t> rows(std::max<int64_t>(in->nnz, 1));
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = in->rowptr[i]; e < in->rowptr[i + 1]; ++e) rows[e] = (int32_t)i;
    DevBuf<int32_t> drows;
    DevBuf<double> sv;
    drows.reserve(rows.size());
    sv.reserve(rows.size());
    SIC_HIP(hipMemcpyAsync(drows.p, rows.data(), sizeof(int32_t) * in->nnz, hipMemcpyHostToDevice, s));
    launch_sddmm(P.Xt.p, P.m, drows.p, A.col.p, in->nnz, sv.p, s);
    std::vector<double> svh(rows.size());
    SIC_HIP(hipMemcpyAsync(svh.data(), sv.p, sizeof(double) * in->nnz, hipMemcpyDeviceToHost, s));
    sync(C);
    double logdet = 0.0;
    for (int t = 0; t < tiles; ++t) {
        if (o[2 * t + 1] == 0.0)
            throw SicError(SIC_ENOTPD, "warm start is not positive definite");
        logdet += o[2 * t];
    }
    double tr = 0.0;
    for (int64_t e = 0; e < in->nnz; ++e) tr += svh[e] * in->val[e];
    return -logdet + tr + P.lam * l1;
}

void relabel_csr(int64_t n, const std::vector<int64_t>& rp, const std::vector<int32_t>& cl,
                 const std::vector<double>& vl, const std::vector<int32_t>& map,
                 int64_t* brp, int32_t* bcl, double* bvl);

void get_A_host(Context& C, Problem& P, sic_csr* out) {
    DevCSR& A = P.Acur();
    const int64_t n = P.n, nnz = A.nnz;
    out->n = n;
    out->nnz = nnz;
    out->rowptr = (int64_t*)malloc(sizeof(int64_t) * (n + 1));
    out->col = (int32_t*)malloc(sizeof(int32_t) * std::max<int64_t>(nnz, 1));
    out->val = (double*)malloc(sizeof(double) * std::max<int64_t>(nnz, 1));
    if (!out->rowptr || !out->col || !out->val) {
        free(out->rowptr); free(out->col); free(out->val);
        out->rowptr = nullptr; out->col = nullptr; out->val = nullptr;
        throw SicError(SIC_ENOMEM, "host allocation for the result failed");
    }
    SIC_HIP(hipMemcpyAsync(out->rowptr, A.rowptr.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, C.stream));
    if (nnz) {
        SIC_HIP(hipMemcpyAsync(out->col, A.col.p, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, C.stream));
        SIC_HIP(hipMemcpyAsync(out->val, A.val.p, sizeof(double) * nnz, hipMemcpyDeviceToHost, C.stream));
    }
    sync(C);
    if (!P.perm.empty()) {
        // back to the caller's labels: row perm[p] holds row p, columns relabelled
        std::vector<int64_t> rp(out->rowptr, out->rowptr + n + 1);
        std::vector<int32_t> cl(out->col, out->col + nnz);
        std::vector<double> vl(out->val, out->val + nnz);
        relabel_csr(n, rp, cl, vl, P.perm, out->rowptr, out->col, out->val);
    }
}

// B = the symmetric CSR (rp, cl, vl) with every label p renamed to = map[p]:
// row map[p] of B is row p of the input, its columns renamed and sorted.
void relabel_csr(int64_t n, const std::vector<int64_t>& rp, const std::vector<int32_t>& cl,
                 const std::vector<double>& vl, const std::vector<int32_t>& map,
                 int64_t* brp, int32_t* bcl, double* bvl) {
    std::vector<int32_t> inv(n);
    for (int64_t p = 0; p < n; ++p) inv[map[p]] = (int32_t)p;
    brp[0] = 0;
    for (int64_t r = 0; r < n; ++r) brp[r + 1] = brp[r] + (rp[inv[r] + 1] - rp[inv[r]]);
    std::vector<std::pair<int32_t, double>> row;
    for (int64_t r = 0; r < n; ++r) {
        const int64_t p = inv[r];
        row.clear();
        for (int64_t e = rp[p]; e < rp[p + 1]; ++e) row.emplace_back(map[cl[e]], vl[e]);
        std::sort(row.begin(), row.end());
        int64_t o = brp[r];
        for (const auto& x : row) {
            bcl[o] = x.first;
            bvl[o] = x.second;
            ++o;
        }
    }
}

void set_level_keys(Context& C, Problem& P, const int64_t* keys, int64_t count) {
    const int64_t n = P.n;
    std::vector<int64_t> cnt(n + 1, 0);
    for (int64_t t = 0; t < count; ++t) {
        const int64_t i = keys[t] / n, j = keys[t] % n;
        if (i < 0 || j < 0 || i >= n || j >= n || i > j)
            throw SicError(SIC_EINVAL, "level key out of range (expects i*n+j with i <= j)");
        cnt[i + 1]++;
        if (i != j) cnt[j + 1]++;
    }
    for (int64_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    const int64_t total = cnt[n];
    std::vector<int32_t> col(std::max<int64_t>(total, 1));
    std::vector<int64_t> pos(cnt.begin(), cnt.end() - 1);
    for (int64_t t = 0; t < count; ++t) {
        const int64_t i = keys[t] / n, j = keys[t] % n;
        col[pos[i]++] = (int32_t)j;
        if (i != j) col[pos[j]++] = (int32_t)i;
    }
    for (int64_t i = 0; i < n; ++i) {
        std::sort(col.begin() + cnt[i], col.begin() + cnt[i + 1]);
        auto last = std::unique(col.begin() + cnt[i], col.begin() + cnt[i + 1]);
        if (last != col.begin() + cnt[i + 1]) throw SicError(SIC_EINVAL, "duplicate level keys");
    }
    P.crow.reserve(n + 1);
    P.ccol.reserve(std::max<int64_t>(total, 1));
    SIC_HIP(hipMemcpyAsync(P.crow.p, cnt.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, C.stream));
    if (total)
        SIC_HIP(hipMemcpyAsync(P.ccol.p, col.data(), sizeof(int32_t) * total, hipMemcpyHostToDevice, C.stream));
    sync(C);
    P.crow_h = std::move(cnt);
    P.level_set = true;
}

// ------------------------------------------------------------------ one block

// Step (d) on the coordinates prepared in the block work area: the explicit
// coordinate Hessian form when the block has at most cd_hessian_max
// coordinates (and its z and Delta fit in LDS), else the U = Delta W form.
// Returns the profiler record to scale by the sweep count (or -1).
// S_J of columns [j0, j0+b) in the current sweep's precision (float64 result).
static void cov_block(Context& C, Problem& P, int64_t j0, int b, double* out, hipStream_t st) {
    const size_t n = (size_t)P.n, w = sizeof(double) * (size_t)b;
    if (P.scache) {
        // With the cache every column is formed once, in float64 whatever the
        // cycle's precision, and copied out afterwards (the same kernel on the
        // same samples: the same values); the reduced-precision products run
        // only without it.
        if (!std::all_of(P.s_cached.begin() + j0, P.s_cached.begin() + j0 + b,
                         [](char c) { return c != 0; })) {
            launch_sj_gemm_f64(P.X.p, P.n, P.m, j0, b, out, st);
            SIC_HIP(hipMemcpy2DAsync(P.Scache.p + j0, sizeof(double) * n, out, w, w, n,
                                     hipMemcpyDeviceToDevice, st));
            std::fill(P.s_cached.begin() + j0, P.s_cached.begin() + j0 + b, 1);
            return;
        }
        SIC_HIP(hipMemcpy2DAsync(out, w, P.Scache.p + j0, sizeof(double) * n, w, n,
                                 hipMemcpyDeviceToDevice, st));
        return;
    }
    if (C.prec != PREC_F64 && P.narrow)
        launch_sj_gemm_low(C.prec == PREC_BF16 ? (const void*)P.Xb.p : (const void*)P.Xf.p,
                           C.prec == PREC_BF16, P.n, P.m, j0, b, out, st);
    else
        launch_sj_gemm_f64(P.X.p, P.n, P.m, j0, b, out, st);
}

// The sweep statistics (8 doubles), written by the CD kernels straight into
// pinned staging.
static double* cd_stats(Context& C) { return C.h_f64 + 40; }

static int64_t run_cd(Context& C, int jp, int b, int64_t nc, double lam, int max_sweeps,
                      double tol) {
    BlockWork& W = C.work;
    hipStream_t s = C.stream;
    double* stats = cd_stats(C);
    if (nc > 0 && C.opt.pcd_min_coords > 0 && nc >= C.opt.pcd_min_coords)
        return launch_pcd(nc, jp, b, W.cptr.p, W.c_p.p, W.c_ci.p, W.c_S.p, W.c_A.p, W.c_wtc.p,
                          W.c_inva.p, W.WJJ.p, lam, 10 * max_sweeps, tol, W.delta.p,
                          W.pcd, stats, C.h_f64 + 32, s);
    if (nc > 0 && nc <= C.opt.cd_hessian_max && nc <= cd_hessian_limit() &&
        cd_hessian_lds_bytes(nc) <= CD_MAX_LDS_BYTES) {
        W.HT.reserve((size_t)nc * nc);
        W.cdx.reserve(cd_exchange_doubles());
        return launch_cd_hessian(nc, jp, W.c_p.p, W.c_ci.p, W.WJJ.p, W.c_S.p, W.c_A.p,
                                 W.c_inva.p, W.c_wtc.p, lam, max_sweeps, tol, W.HT.p, W.delta.p,
                                 stats, W.cdx.p, s, C.prec != PREC_F64);
    }
    W.U.reserve((size_t)jp * b);
    W.ug.reserve(jp);
    W.markg.reserve(jp);
    SIC_HIP(hipMemsetAsync(W.U.p, 0, sizeof(double) * jp * b, s));
    launch_cd(jp, b, W.cptr.p, W.c_p.p, W.c_S.p, W.c_A.p, W.c_inva.p, W.c_wtc.p, W.WJJ.p, lam,
              max_sweeps, tol, W.U.p, W.delta.p, W.mu.p, W.ug.p, W.markg.p, stats, s);
    return -1;
}

static BlockResult block_update_body(Context& C, Problem& P, int64_t j0, int b, bool fine,
                                     bool record, double tolI, double tolN) {
    hipStream_t s = C.stream;
    BlockWork& W = C.work;
    const int64_t n = P.n;
    DevCSR& A = P.Acur();
    if (!fine && !P.level_set) throw SicError(SIC_EINVAL, "coarse block without a level set");
    ensure_flags(C, n, b);
    BlockResult R;
    R.j0 = j0;
    R.b = b;
    R.level = fine ? 0 : 1;
    const size_t nb = (size_t)n * b;
    W.AJ.reserve(nb);
    SIC_HIP(hipMemsetAsync(W.AJ.p, 0, sizeof(double) * nb, s));
    launch_scatter_aj(A, j0, b, W.AJ.p, s);
    W.colptr.reserve(b + 1);
    W.ccount.reserve(b);
    W.kkt_acc.reserve(2);
    int64_t nC = 0;
    if (fine) {
        // (a) S_J on the side stream (it reads X only) beside (b) W_I by CG on
        // the main one, then (c) screening over all rows once both are done
        W.SJ.reserve(nb);
        W.WI.reserve(nb);
        W.cols.reserve(std::max<int64_t>(b, 1));
        SIC_HIP(hipEventRecord(C.ev_fork, s));
        SIC_HIP(hipStreamWaitEvent(C.side, C.ev_fork, 0));
        cov_block(C, P, j0, b, W.SJ.p, C.side);
        SIC_HIP(hipEventRecord(C.ev_join, C.side));
        launch_iota_i32(W.cols.p, b, (int32_t)j0, s);
        CGResult cg = block_cg(A, W.cols.p, b, W.WI.p, b, tolI, C.opt.cg_max_iter, W.cg, s,
                               C.prec != PREC_F64, 0, P.warm_store());
        check_cg(cg, "W_I");
        R.cg_iters_I = cg.iterations;
        R.cg_res_I = cg.max_rel_res;
        SIC_HIP(hipStreamWaitEvent(s, C.ev_join, 0));
        const int tiles = (int)((n + ROWS_PER_TILE - 1) / ROWS_PER_TILE);
        W.tilecount.reserve((size_t)tiles * b);
        W.offsets.reserve((size_t)tiles * b);
        W.kkt.reserve(2 * (size_t)tiles);
        launch_screen_fine(0, n, j0, b, ROWS_PER_TILE, tiles, P.lam, W.SJ.p, W.WI.p, W.AJ.p,
                           W.tilecount.p, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                           W.nflag.p, W.kkt.p, s);
        if (record) launch_kkt_accumulate(W.kkt.p, tiles, W.kkt_acc.p, s);
        launch_scan_colmajor(W.tilecount.p, tiles, b, W.offsets.p, W.colptr.p, C.h_i64 + 2, s);
        reserve_free_lists(W, nb);
        launch_screen_fine(1, n, j0, b, ROWS_PER_TILE, tiles, P.lam, W.SJ.p, W.WI.p, W.AJ.p,
                           W.tilecount.p, W.offsets.p, W.e_row.p, W.e_g.p, W.e_s.p, W.e_a.p,
                           W.e_w.p, W.nflag.p, W.kkt.p, s);
    } else {
        // coarse level: candidates C_l of the block columns, S by sampled dot
        // products, W_{N^C} by CG and W_II by the neighbour identity (App. A.2)
        const int64_t base = P.crow_h[j0];
        const int64_t cnt = P.crow_h[j0 + b] - base;
        W.cand_col.reserve(std::max<int64_t>(cnt, 1));
        W.S_cand.reserve(std::max<int64_t>(cnt, 1));
        // A_II = L L^T on the side stream (it reads A only) beside the candidate
        // products and the W_{N^C} conjugate gradient
        const size_t bb = (size_t)b * b;
        W.Kb.reserve(bb); W.AII.reserve(bb); W.WII.reserve(bb); W.Dinv.reserve(8 * 1024);
        W.err.reserve(1);
        double* h = C.h_f64 + 48;   // A_II's log det and PD flag, written by the factor
        SIC_HIP(hipEventRecord(C.ev_fork, s));
        SIC_HIP(hipStreamWaitEvent(C.side, C.ev_fork, 0));
        launch_dense_aii(A, j0, b, W.AII.p, C.side);
        launch_chol(W.AII.p, (int64_t)bb, 1, b, b, 0, h, C.side, W.Dinv.p);
        launch_zero_upper(W.AII.p, b, b, C.side);
        SIC_HIP(hipEventRecord(C.ev_join, C.side));
        launch_expand_cand(P.crow.p, j0, b, base, W.cand_col.p, s);
        launch_sddmm(P.Xt.p, P.m, P.ccol.p + base, W.cand_col.p, cnt, W.S_cand.p, s);
        launch_flag_cand(P.ccol.p, base, cnt, j0, b, W.cflag.p, s);
        W.scan_n.reserve(n + 1);
        launch_scan_i32(W.cflag.p, n, W.scan_n.p, C.h_i64 + 3, s);
        sync(C);
        nC = C.h_i64[3];
        R.nC = nC;
        W.NC.reserve(std::max<int64_t>(nC, 1));
        launch_flag_compact(W.cflag.p, W.scan_n.p, n, W.NC.p, W.cmap.p, s);
        W.WNC.reserve((size_t)n * std::max<int64_t>(nC, 1));
        if (nC > 0) {
            CGResult cg = block_cg(A, W.NC.p, (int)nC, W.WNC.p, nC, tolI, C.opt.cg_max_iter, W.cg,
                                   s, C.prec != PREC_F64, 2, P.warm_store());
            check_cg(cg, "W_{N^C}");
            R.cg_iters_N = cg.iterations;
            R.cg_res_N = cg.max_rel_res;
        }
        SIC_HIP(hipMemsetAsync(W.err.p, 0, sizeof(int32_t), s));
        launch_a2_k(A, j0, b, W.WNC.p, nC, W.cmap.p, W.Kb.p, W.err.p, s);
        launch_identity_minus(W.Kb.p, b, W.WII.p, s);
        SIC_HIP(hipStreamWaitEvent(s, C.ev_join, 0));
        launch_trsm_lower(W.AII.p, b, b, W.Dinv.p, W.WII.p, b, b, 0, s);
        launch_trsm_lower(W.AII.p, b, b, W.Dinv.p, W.WII.p, b, b, 1, s);
        int32_t* herr = reinterpret_cast<int32_t*>(C.h_i64 + 16);
        SIC_HIP(hipMemcpyAsync(herr, W.err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        sync(C);
        if (*herr) throw SicError(SIC_EINTERNAL, "support of A is not inside the level set");
        if (h[1] == 0.0) throw SicError(SIC_ENOTPD, "diagonal block of A is not positive definite");
        launch_screen_coarse(0, P.crow.p, P.ccol.p, base, j0, b, P.lam, W.S_cand.p, W.WII.p,
                             W.WNC.p, nC, W.cmap.p, W.AJ.p, W.ccount.p, nullptr, nullptr, nullptr,
                             nullptr, nullptr, nullptr, W.nflag.p, s);
        launch_scan_i32(W.ccount.p, b, W.colptr.p, C.h_i64 + 2, s);
        reserve_free_lists(W, nb);
        launch_screen_coarse(1, P.crow.p, P.ccol.p, base, j0, b, P.lam, W.S_cand.p, W.WII.p,
                             W.WNC.p, nC, W.cmap.p, W.AJ.p, W.ccount.p, W.colptr.p, W.e_row.p,
                             W.e_g.p, W.e_s.p, W.e_a.p, W.e_w.p, W.nflag.p, s);
    }
    // neighbourhood N and J' = I u N, and the coordinates; |N| and the
    // coordinate count come back in one read (J' is sized for b + n, past any
    // count the flags can give)
    W.scan_n.reserve(n + 1);
    launch_scan_i32(W.nflag.p, n, W.scan_n.p, C.h_i64, s);
    W.Jp.reserve(n + b);
    launch_nbr_compact(W.nflag.p, W.scan_n.p, n, j0, b, W.Jp.p, W.lmap.p, s);
    W.cptr.reserve(b + 1);
    launch_coord_count(W.colptr.p, W.e_row.p, j0, b, W.ccount.p, s);
    launch_scan_i32(W.ccount.p, b, W.cptr.p, C.h_i64 + 1, s);
    // |N|, the coordinate count and E = colptr[b] were written by the scans
    // straight into pinned staging
    sync(C);
    R.nN = C.h_i64[0];
    R.ncoord = C.h_i64[1];
    R.E = C.h_i64[2];
    const int64_t nN = R.nN;
    const int64_t jp64 = b + nN;
    if (jp64 > (int64_t)INT32_MAX / 2) throw SicError(SIC_ETOOBIG, "neighbourhood too large");
    const int jp = (int)jp64;
    R.jp = jp;
    const int64_t nc = R.ncoord;
    const size_t ncs = (size_t)std::max<int64_t>(nc, 1);
    W.c_p.reserve(ncs); W.c_e.reserve(ncs); W.c_ci.reserve(ncs);
    W.c_S.reserve(ncs); W.c_A.reserve(ncs); W.c_a.reserve(ncs); W.c_inva.reserve(ncs);
    W.c_wtc.reserve(ncs); W.c_wtt.reserve(ncs); W.delta.reserve(ncs); W.mu.reserve(ncs);
    launch_coord_fill(W.colptr.p, W.e_row.p, W.e_s.p, W.e_a.p, W.cptr.p, W.lmap.p, j0, b, W.c_p.p,
                      W.c_e.p, W.c_S.p, W.c_A.p, s);
    // W_N at the finest level
    if (fine && nN > 0) {
        W.WN.reserve((size_t)n * nN);
        CGResult cg = block_cg(A, W.Jp.p + b, (int)nN, W.WN.p, nN, tolN, C.opt.cg_max_iter, W.cg,
                               s, C.prec != PREC_F64, 1, P.warm_store());
        check_cg(cg, "W_N");
        R.cg_iters_N = cg.iterations;
        R.cg_res_N = cg.max_rel_res;
    }
    // W on J' x J'
    W.WJJ.reserve((size_t)jp * jp);
    launch_gather_wjj(fine ? 0 : 1, W.Jp.p, jp, b, W.WI.p, W.WN.p, nN, W.WII.p, W.WNC.p, nC,
                      W.cmap.p, W.WJJ.p, s);
    // W_II = R R^T for the line search on the side stream, beside the
    // coordinate descent (one workgroup each): the side stream starts once W_J'J'
    // is gathered, the line search waits for it
    ls_reserve(C, b, nN);
    SIC_HIP(hipEventRecord(C.ev_fork, s));
    SIC_HIP(hipStreamWaitEvent(C.side, C.ev_fork, 0));
    ls_factor_wii(C, jp, b, C.side);
    SIC_HIP(hipEventRecord(C.ev_join, C.side));
    // (d) coordinate descent
    launch_cd_prep(W.cptr.p, b, nc, W.c_p.p, W.WJJ.p, jp, W.c_ci.p, W.c_a.p, W.c_inva.p, W.c_wtc.p,
                   W.c_wtt.p, W.delta.p, s);
    if (fine && C.prec != PREC_F64 && nc > 0) {
        // reduced-precision S_J served the screening; the model the direction
        // and the line search use takes float64 S at its coordinates (a
        // sampled product of 2 m flops each, against 2 n b m for the block)
        W.c_gr.reserve(ncs);
        W.c_gc.reserve(ncs);
        launch_coord_globals(nc, W.c_p.p, W.c_ci.p, W.Jp.p, j0, W.c_gr.p, W.c_gc.p, s);
        launch_sddmm(P.Xt.p, P.m, W.c_gr.p, W.c_gc.p, nc, W.c_S.p, s);
    }
    const int64_t cd_rec = run_cd(C, jp, b, nc, P.lam, C.opt.cd_max_sweeps, C.opt.cd_tol);
    // the sweep statistics are in pinned staging once the line search's first
    // read-back has waited for the stream
    const double* h_cds = cd_stats(C);
    // (e) line search
    LineSearch ls = line_search(C, P.lam, jp, b, nN, nc, true);   // ends on its read-back
    double cds[8];
    std::copy(h_cds, h_cds + 8, cds);
    if (cds[7] != 0.0) throw SicError(SIC_EINTERNAL, "CD sweep workgroups timed out waiting on one another");
    R.cd_sweeps = (int)cds[0];
    R.cd_last_maxmu = cds[1];
    prof_scale(cd_rec, cds[0]);
    if (C.opt.flags & SIC_FLAG_VERBOSE)
        fprintf(stderr,
                "[sic] block j0=%lld %s E=%lld coords=%lld |N|=%lld |NC|=%lld cg=%d/%d cd=%d "
                "cd-clocks(us) %.0f/%.0f/%.0f/%.0f alpha=%g trials=%d\n",
                (long long)j0, fine ? "fine" : "coarse", (long long)R.E, (long long)nc,
                (long long)nN, (long long)nC, R.cg_iters_I, R.cg_iters_N, R.cd_sweeps,
                cds[3] / 100.0, cds[4] / 100.0, cds[5] / 100.0, cds[6] / 100.0, ls.alpha,
                ls.trials);
    if (!ls.wii_pd) throw SicError(SIC_EINTERNAL, "W_II is not positive definite (inaccurate inverse columns)");
    R.alpha = ls.alpha;
    R.dF = ls.dF;
    R.trials = ls.trials;
    // A <- A + alpha Delta
    bool new_nnz_pending = false;
    int64_t new_cap = 0;
    if (ls.alpha != 0.0) {
        DevCSR& An = P.A[1 - P.cur];
        const int64_t cap = A.nnz + 2 * nc;
        An.n = n;
        An.rowptr.reserve(n + 1);
        An.col.reserve_grow(std::max<int64_t>(cap, 1));
        An.val.reserve_grow(std::max<int64_t>(cap, 1));
        W.rcount.reserve(n);
        launch_upd_newvals(nc, W.c_p.p, W.c_ci.p, W.c_A.p, W.delta.p, ls.alpha, W.Jp.p, j0, b,
                           W.ANEW.p, s);
        launch_upd_rows(0, n, j0, b, A, W.lmap.p, W.cptr.p, W.c_p.p, W.Jp.p, W.ANEW.p, W.rcount.p,
                        nullptr, nullptr, nullptr, s);
        // the new entry count goes straight to pinned staging, read at the block's
        // closing synchronisation; the fill pass writes nothing at or beyond cap
        launch_scan_i32(W.rcount.p, n, An.rowptr.p, C.h_i64 + 8, s);
        new_nnz_pending = true;
        new_cap = cap;
        launch_upd_rows(1, n, j0, b, A, W.lmap.p, W.cptr.p, W.c_p.p, W.Jp.p, W.ANEW.p, W.rcount.p,
                        An.rowptr.p, An.col.p, An.val.p, s, cap);
        launch_upd_reset(nc, W.c_p.p, W.c_ci.p, W.Jp.p, j0, b, W.ANEW.p, s);
        P.cur = 1 - P.cur;
        P.F += ls.dF;
    }
    // free pairs and |g| for the next hierarchy: copied to pinned memory here,
    // recorded after the block's closing synchronisation
    const bool rec = record && R.E > 0;
    if (rec) {
        W.h_cp.reserve_grow(b + 1);
        W.h_rows.reserve_grow(R.E);
        W.h_g.reserve_grow(R.E);
        SIC_HIP(hipMemcpyAsync(W.h_cp.p, W.colptr.p, sizeof(int64_t) * (b + 1), hipMemcpyDeviceToHost, s));
        SIC_HIP(hipMemcpyAsync(W.h_rows.p, W.e_row.p, sizeof(int32_t) * R.E, hipMemcpyDeviceToHost, s));
        SIC_HIP(hipMemcpyAsync(W.h_g.p, W.e_g.p, sizeof(double) * R.E, hipMemcpyDeviceToHost, s));
    }
    // reset per-block flags and maps
    SIC_HIP(hipMemsetAsync(W.nflag.p, 0, sizeof(int32_t) * n, s));
    launch_reset_rows(W.Jp.p, jp, nullptr, W.lmap.p, s);
    if (!fine && nC > 0) launch_reset_rows(W.NC.p, nC, W.cflag.p, W.cmap.p, s);
    sync(C);
    if (rec) {
        const int64_t* cp = W.h_cp.p;
        const int32_t* rows = W.h_rows.p;
        const double* g = W.h_g.p;
        int64_t seq = (int64_t)P.rec_seq.size();
        for (int ci = 0; ci < b; ++ci) {
            const int64_t c = j0 + ci;
            for (int64_t e = cp[ci]; e < cp[ci + 1]; ++e) {
                const int64_t r = rows[e];
                const int64_t key = r <= c ? r * n + c : c * n + r;
                P.rec_key.push_back(key);
                P.rec_g.push_back(std::fabs(g[e]));
                P.rec_seq.push_back(seq++);
            }
        }
    }
    if (new_nnz_pending) {
        DevCSR& An = P.Acur();
        An.nnz = C.h_i64[8];
        if (An.nnz > new_cap) throw SicError(SIC_EINTERNAL, "CSR rebuild exceeded its bound");
        P.max_nnz = std::max(P.max_nnz, An.nnz);
    }
    R.nnz_after = P.Acur().nnz;
    C.last = R;
    return R;
}

BlockResult block_update(Context& C, Problem& P, int64_t j0, int b, bool fine, bool record,
                         double tolI, double tolN) {
    try {
        return block_update_body(C, P, j0, b, fine, record, tolI, tolN);
    } catch (...) {
        // an abandoned block leaves its row flags and maps set: the next block
        // update clears them all again
        C.work.n_init = 0;
        throw;
    }
}

// ------------------------------------------------------------------ sweeps

static void finish_records(Problem& P) {
    const size_t N = P.rec_key.size();
    std::vector<size_t> idx(N);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](size_t a, size_t b) {
        if (P.rec_key[a] != P.rec_key[b]) return P.rec_key[a] < P.rec_key[b];
        return P.rec_seq[a] < P.rec_seq[b];
    });
    std::vector<int64_t> k;
    std::vector<double> g;
    k.reserve(N);
    g.reserve(N);
    for (size_t t = 0; t < N; ++t) {
        const size_t i = idx[t];
        if (t + 1 < N && P.rec_key[idx[t + 1]] == P.rec_key[i]) continue;   // keep the latest
        k.push_back(P.rec_key[i]);
        g.push_back(P.rec_g[i]);
    }
    P.rec_key = std::move(k);
    P.rec_g = std::move(g);
    P.rec_seq.clear();
}

void initial_free_set(Context& C, Problem& P) {
    // W = A^{-1} = I at A = I: free pairs are |S_ij| > lambda plus the diagonal
    hipStream_t s = C.stream;
    BlockWork& W = C.work;
    const int64_t n = P.n;
    const int b = (int)std::min<int64_t>(C.opt.block, n);
    ensure_flags(C, n, b);
    P.rec_key.clear();
    P.rec_g.clear();
    P.rec_seq.clear();
    W.kkt_acc.reserve(2);
    const int tiles = (int)((n + ROWS_PER_TILE - 1) / ROWS_PER_TILE);
    // the block-sized buffers at the largest (first) block's size up front: none
    // is reallocated while the stream may still read it
    W.SJ.reserve((size_t)n * b);
    W.AJ.reserve((size_t)n * b);
    W.colptr.reserve(b + 1);
    W.tilecount.reserve((size_t)tiles * b);
    W.offsets.reserve((size_t)tiles * b);
    W.kkt.reserve(2 * (size_t)tiles);
    // count pass of a block: S_J and A_J, then the free pairs per (tile, column)
    // and their total, which the scan writes straight into pinned staging
    auto count_pairs = [&](int64_t j0, int bb) {
        SIC_HIP(hipMemsetAsync(W.AJ.p, 0, sizeof(double) * (size_t)n * bb, s));
        launch_scatter_aj(P.Acur(), j0, bb, W.AJ.p, s);
        cov_block(C, P, j0, bb, W.SJ.p, s);
        launch_screen_fine(0, n, j0, bb, ROWS_PER_TILE, tiles, P.lam, W.SJ.p, nullptr, W.AJ.p,
                           W.tilecount.p, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                           W.nflag.p, W.kkt.p, s);
        launch_scan_colmajor(W.tilecount.p, tiles, bb, W.offsets.p, W.colptr.p, C.h_i64, s);
    };
    // block k's pairs come back into pinned slot k % 2; the host records them
    // while the stream screens block k + 1
    HostBuf<int64_t>* h_cp[2] = {&W.h_cp, &W.h_cp_alt};
    HostBuf<int32_t>* h_rows[2] = {&W.h_rows, &W.h_rows_alt};
    HostBuf<double>* h_g[2] = {&W.h_g, &W.h_g_alt};
    struct Pending { int64_t j0 = 0; int bb = 0; int q = 0; bool on = false; } pend;
    auto record_pairs = [&](const Pending& pd) {
        const int64_t* cp = h_cp[pd.q]->p;
        const int32_t* rows = h_rows[pd.q]->p;
        const double* g = h_g[pd.q]->p;
        int64_t seq = (int64_t)P.rec_seq.size();
        for (int ci = 0; ci < pd.bb; ++ci) {
            const int64_t c = pd.j0 + ci;
            for (int64_t e = cp[ci]; e < cp[ci + 1]; ++e) {
                const int64_t r = rows[e];
                const int64_t key = r <= c ? r * n + c : c * n + r;
                P.rec_key.push_back(key);
                P.rec_g.push_back(std::fabs(g[e]));
                P.rec_seq.push_back(seq++);
            }
        }
    };
    const int64_t nblocks = (n + b - 1) / b;
    count_pairs(0, b);
    for (int64_t k = 0; k < nblocks; ++k) {
        const int64_t j0 = k * b;
        const int bb = (int)std::min<int64_t>(b, n - j0);
        // block k is counted, and block k - 1's pairs are in their pinned slot;
        // nothing is queued on the stream here
        sync(C);
        const int64_t E = C.h_i64[0];
        const size_t Es = (size_t)std::max<int64_t>(E, 1);
        W.e_row.reserve(Es); W.e_g.reserve(Es); W.e_s.reserve(Es); W.e_a.reserve(Es); W.e_w.reserve(Es);
        const int q = (int)(k & 1);
        h_cp[q]->reserve_grow(bb + 1);
        h_rows[q]->reserve_grow(Es);
        h_g[q]->reserve_grow(Es);
        launch_screen_fine(1, n, j0, bb, ROWS_PER_TILE, tiles, P.lam, W.SJ.p, nullptr, W.AJ.p,
                           W.tilecount.p, W.offsets.p, W.e_row.p, W.e_g.p, W.e_s.p, W.e_a.p,
                           W.e_w.p, W.nflag.p, W.kkt.p, s);
        SIC_HIP(hipMemcpyAsync(h_cp[q]->p, W.colptr.p, sizeof(int64_t) * (bb + 1), hipMemcpyDeviceToHost, s));
        SIC_HIP(hipMemcpyAsync(h_rows[q]->p, W.e_row.p, sizeof(int32_t) * Es, hipMemcpyDeviceToHost, s));
        SIC_HIP(hipMemcpyAsync(h_g[q]->p, W.e_g.p, sizeof(double) * Es, hipMemcpyDeviceToHost, s));
        SIC_HIP(hipMemsetAsync(W.nflag.p, 0, sizeof(int32_t) * n, s));
        if (k + 1 < nblocks) count_pairs(j0 + b, (int)std::min<int64_t>(b, n - j0 - b));
        if (pend.on) record_pairs(pend);
        pend = Pending{j0, bb, q, true};
    }
    sync(C);
    if (pend.on) record_pairs(pend);
    finish_records(P);
}

SweepResult sweep(Context& C, Problem& P, bool fine, double tolI, double tolN) {
    SweepResult S;
    const int64_t n = P.n;
    const int b = (int)std::min<int64_t>(C.opt.block, n);
    if (fine) {
        C.work.kkt_acc.reserve(2);
        SIC_HIP(hipMemsetAsync(C.work.kkt_acc.p, 0, sizeof(double) * 2, C.stream));
        P.rec_key.clear();
        P.rec_g.clear();
        P.rec_seq.clear();
    }
    for (int64_t j0 = 0; j0 < n; j0 += b) {
        const int bb = (int)std::min<int64_t>(b, n - j0);
        BlockResult R = block_update(C, P, j0, bb, fine, fine, tolI, tolN);
        S.cg_iters += R.cg_iters_I + R.cg_iters_N;
        S.cd_sweeps += R.cd_sweeps;
        S.blocks += 1;
    }
    if (fine) {
        double acc[2];
        SIC_HIP(hipMemcpyAsync(acc, C.work.kkt_acc.p, sizeof(double) * 2, hipMemcpyDeviceToHost, C.stream));
        sync(C);
        S.kkt_max = acc[0];
        S.kkt_l1 = acc[1];
        finish_records(P);
    }
    return S;
}

// ------------------------------------------------------------------ hierarchy

void hierarchy_host(int64_t n, const std::vector<int64_t>& supp, const std::vector<int64_t>& fkey,
                    const std::vector<double>& fg, std::vector<int64_t>& ranking,
                    std::vector<int64_t>& sizes) {
    (void)n;
    std::vector<int64_t> sp(supp);
    std::sort(sp.begin(), sp.end());
    sp.erase(std::unique(sp.begin(), sp.end()), sp.end());
    std::vector<size_t> rest;
    rest.reserve(fkey.size());
    for (size_t t = 0; t < fkey.size(); ++t)
        if (!std::binary_search(sp.begin(), sp.end(), fkey[t])) rest.push_back(t);
    std::sort(rest.begin(), rest.end(), [&](size_t a, size_t b) {
        if (fg[a] != fg[b]) return fg[a] > fg[b];
        return fkey[a] < fkey[b];
    });
    ranking = sp;
    for (size_t t : rest) ranking.push_back(fkey[t]);
    const int64_t nf = (int64_t)ranking.size(), ns = (int64_t)sp.size();
    sizes.clear();
    sizes.push_back(std::max((nf + 1) / 2, ns));
    while (sizes.back() != ns) sizes.push_back(std::max((sizes.back() + 1) / 2, ns));
}

std::vector<int64_t> support_keys(Context& C, Problem& P) {
    DevCSR& A = P.Acur();
    const int64_t n = P.n;
    std::vector<int64_t> rp(n + 1);
    std::vector<int32_t> cl(std::max<int64_t>(A.nnz, 1));
    SIC_HIP(hipMemcpyAsync(rp.data(), A.rowptr.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, C.stream));
    SIC_HIP(hipMemcpyAsync(cl.data(), A.col.p, sizeof(int32_t) * A.nnz, hipMemcpyDeviceToHost, C.stream));
    sync(C);
    std::vector<int64_t> keys;
    keys.reserve(A.nnz / 2 + n);
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rp[i]; e < rp[i + 1]; ++e)
            if (cl[e] >= i) keys.push_back(i * n + cl[e]);
    return keys;   // ascending: rows ascending, columns sorted
}

void cluster_problem(Context& C, Problem& P) {
    hipStream_t s = C.stream;
    const int64_t n = P.n, m = P.m;
    const int b = (int)std::min<int64_t>(C.opt.block, n);
    std::vector<int64_t> keys = support_keys(C, P);
    keys.insert(keys.end(), P.rec_key.begin(), P.rec_key.end());
    const std::vector<int32_t> order = cluster_order(n, keys.data(), (int64_t)keys.size(), b);
    bool same = true;
    for (int64_t p = 0; p < n && same; ++p) same = order[p] == p;
    if (same) return;
    std::vector<int32_t> inv(n);
    for (int64_t p = 0; p < n; ++p) inv[order[p]] = (int32_t)p;
    // samples: column p of the new X is column order[p] of the old one
    BlockWork& W = C.work;
    W.perm.reserve(n);
    SIC_HIP(hipMemcpyAsync(W.perm.p, order.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, s));
    const size_t count = (size_t)n * m;
    W.xstage.reserve(count * sizeof(double));
    launch_gather_cols(P.X.p, m, n, W.perm.p, reinterpret_cast<double*>(W.xstage.p), s);
    SIC_HIP(hipMemcpyAsync(P.X.p, W.xstage.p, count * sizeof(double), hipMemcpyDeviceToDevice, s));
    launch_transpose(P.X.p, m, n, P.Xt.p, s);
    launch_diag_s(P.Xt.p, n, m, P.diagS.p, s);
    if (P.narrow) launch_narrow(P.X.p, (int64_t)count, P.Xf.p, P.Xb.p, s);
    // the iterate, relabelled on the host
    DevCSR& A = P.Acur();
    const int64_t nnz = A.nnz;
    std::vector<int64_t> rp(n + 1), nrp(n + 1);
    std::vector<int32_t> cl(std::max<int64_t>(nnz, 1)), ncl(std::max<int64_t>(nnz, 1));
    std::vector<double> vl(std::max<int64_t>(nnz, 1)), nvl(std::max<int64_t>(nnz, 1));
    SIC_HIP(hipMemcpyAsync(rp.data(), A.rowptr.p, sizeof(int64_t) * (n + 1), hipMemcpyDeviceToHost, s));
    SIC_HIP(hipMemcpyAsync(cl.data(), A.col.p, sizeof(int32_t) * nnz, hipMemcpyDeviceToHost, s));
    SIC_HIP(hipMemcpyAsync(vl.data(), A.val.p, sizeof(double) * nnz, hipMemcpyDeviceToHost, s));
    sync(C);
    relabel_csr(n, rp, cl, vl, inv, nrp.data(), ncl.data(), nvl.data());
    SIC_HIP(hipMemcpyAsync(A.rowptr.p, nrp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, s));
    SIC_HIP(hipMemcpyAsync(A.col.p, ncl.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice, s));
    SIC_HIP(hipMemcpyAsync(A.val.p, nvl.data(), sizeof(double) * nnz, hipMemcpyHostToDevice, s));
    // recorded free pairs
    std::vector<std::pair<int64_t, double>> rec(P.rec_key.size());
    for (size_t t = 0; t < P.rec_key.size(); ++t) {
        const int64_t i = inv[P.rec_key[t] / n], j = inv[P.rec_key[t] % n];
        rec[t] = {i <= j ? i * n + j : j * n + i, P.rec_g[t]};
    }
    std::sort(rec.begin(), rec.end());
    for (size_t t = 0; t < rec.size(); ++t) {
        P.rec_key[t] = rec[t].first;
        P.rec_g[t] = rec[t].second;
    }
    // the caller's label of each new label
    std::vector<int32_t> composed(n);
    for (int64_t p = 0; p < n; ++p) composed[p] = P.perm.empty() ? order[p] : P.perm[order[p]];
    P.perm = std::move(composed);
    P.level_set = false;
    if (P.warm) SIC_HIP(hipMemsetAsync(P.Wvalid.p, 0, (size_t)n, s));   // stored columns: old labels
    std::fill(P.s_cached.begin(), P.s_cached.end(), 0);                  // cached S: old labels
    sync(C);
}

// ------------------------------------------------------------------ exact KKT

static double exact_kkt_body(Context& C, Problem& P, double tol_cg, double* l1) {
    hipStream_t s = C.stream;
    BlockWork& W = C.work;
    const int64_t n = P.n;
    const int b = (int)std::min<int64_t>(C.opt.block, n);
    ensure_flags(C, n, b);
    W.kkt_acc.reserve(2);
    SIC_HIP(hipMemsetAsync(W.kkt_acc.p, 0, sizeof(double) * 2, s));
    for (int64_t j0 = 0; j0 < n; j0 += b) {
        const int bb = (int)std::min<int64_t>(b, n - j0);
        const size_t nb = (size_t)n * bb;
        W.SJ.reserve(nb); W.WI.reserve(nb); W.AJ.reserve(nb);
        W.cols.reserve(bb);
        SIC_HIP(hipMemsetAsync(W.AJ.p, 0, sizeof(double) * nb, s));
        launch_scatter_aj(P.Acur(), j0, bb, W.AJ.p, s);
        launch_sj_gemm_f64(P.X.p, n, P.m, j0, bb, W.SJ.p, s);
        launch_iota_i32(W.cols.p, bb, (int32_t)j0, s);
        check_cg(block_cg(P.Acur(), W.cols.p, bb, W.WI.p, bb, tol_cg, C.opt.cg_max_iter * 4, W.cg,
                          s, false, 3, P.warm_store()),
                 "exact KKT pass");
        const int tiles = (int)((n + ROWS_PER_TILE - 1) / ROWS_PER_TILE);
        W.tilecount.reserve((size_t)tiles * bb);
        W.kkt.reserve(2 * (size_t)tiles);
        launch_screen_fine(0, n, j0, bb, ROWS_PER_TILE, tiles, P.lam, W.SJ.p, W.WI.p, W.AJ.p,
                           W.tilecount.p, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr,
                           W.nflag.p, W.kkt.p, s);
        launch_kkt_accumulate(W.kkt.p, tiles, W.kkt_acc.p, s);
        SIC_HIP(hipMemsetAsync(W.nflag.p, 0, sizeof(int32_t) * n, s));
    }
    double acc[2];
    SIC_HIP(hipMemcpyAsync(acc, W.kkt_acc.p, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
    sync(C);
    if (l1) *l1 = acc[1];
    return acc[0];
}

double exact_kkt(Context& C, Problem& P, double tol_cg, double* l1) {
    try {
        return exact_kkt_body(C, P, tol_cg, l1);
    } catch (...) {
        C.work.n_init = 0;   // row flags of the abandoned pass are cleared again
        throw;
    }
}

// ------------------------------------------------------------------ Algorithm 1

static double a_l1_norm(Context& C, Problem& P) {
    DevCSR& A = P.Acur();
    std::vector<double> v(std::max<int64_t>(A.nnz, 1));
    SIC_HIP(hipMemcpyAsync(v.data(), A.val.p, sizeof(double) * A.nnz, hipMemcpyDeviceToHost, C.stream));
    sync(C);
    double s = 0.0;
    for (int64_t e = 0; e < A.nnz; ++e) s += std::fabs(v[e]);
    return s;
}

// Mixed-precision schedule (reduced precision only while far from the
// optimum): bfloat16 S_J while the last finest sweep's KKT measure exceeds
// 1e-2 (the error of S from bfloat16 samples is ~1e-3), float S_J while it
// exceeds 1e-4 (the CG tolerance is then at least 1e-6, within float CG's
// reach with residual replacement), float64 after that.
static int cycle_precision(const Context& C, const Problem& P, double kkt_prev) {
    if (C.opt.precision != SIC_MIXED || !P.narrow) return PREC_F64;
    if (kkt_prev > 1e-2) return PREC_BF16;
    if (kkt_prev > 1e-4) return PREC_F32;
    return PREC_F64;
}

int solve_problem(Context& C, Problem& P, double tol, sic_info* info) {
    using clk = std::chrono::steady_clock;
    const auto t0 = clk::now();
    auto secs = [&]() { return std::chrono::duration<double>(clk::now() - t0).count(); };
    const bool ml = !(C.opt.flags & SIC_FLAG_NO_MULTILEVEL);
    const bool verbose = (C.opt.flags & SIC_FLAG_VERBOSE) != 0;
    struct PrecReset {   // the step entry points always run in float64
        Context& c;
        ~PrecReset() { c.prec = PREC_F64; }
    } prec_reset{C};
    C.prec = cycle_precision(C, P, INFINITY);
    // continuation (Section 8): lambda_4 = (1 + lambda) / 2 (normalised data puts
    // any useful lambda below 1; never below lambda itself), lambda_3 and
    // lambda_2 linearly spaced towards lambda_1 = lambda, one cycle each, then
    // lambda until convergence. F follows each change of lambda exactly:
    // F changes by (lambda_new - lambda_old) ||A||_1.
    const double lam_target = P.lam;
    const bool cont = (C.opt.flags & SIC_FLAG_CONTINUATION) != 0;
    const double lam4 = std::max(0.5 * (1.0 + lam_target), lam_target);
    auto lam_of = [&](int cyc) {
        return (!cont || cyc >= 3) ? lam_target : lam4 - (lam4 - lam_target) * cyc / 3.0;
    };
    auto set_lambda = [&](double lam) {
        if (lam == P.lam) return;
        P.F += (lam - P.lam) * a_l1_norm(C, P);
        P.lam = lam;
    };
    struct LamReset {   // the solve ends at the caller's lambda whatever happens
        std::function<void()> f;
        ~LamReset() {
            try {
                f();
            } catch (...) {
            }
        }
    } lam_reset{[&]() { set_lambda(lam_target); }};
    set_lambda(lam_of(0));
    initial_free_set(C, P);
    double kkt_prev = INFINITY, kkt_l1 = INFINITY;
    int status = SIC_ENOCONV;
    int cycles = 0, sweeps = 0, trace_len = 0;
    int64_t blocks = 0, cg_it = 0, cd_sw = 0;
    bool certified = false;   // kkt_prev comes from the exact float64 pass
    const bool certify = !(C.opt.flags & SIC_FLAG_NO_CERTIFY);
    const double tol_cert = std::max(1e-13, std::min(1e-10, 0.01 * tol));
    try {
    for (int cyc = 0; cyc < C.opt.max_cycles; ++cyc) {
        const double tolI = std::min(C.opt.cg_tol_I, std::max(1e-12, 0.01 * kkt_prev));
        const double tolN = std::min(C.opt.cg_tol_N, std::max(1e-12, 0.01 * kkt_prev));
        C.prec = cycle_precision(C, P, kkt_prev);
        set_lambda(lam_of(cyc));
        if (C.opt.flags & SIC_FLAG_CLUSTER) cluster_problem(C, P);
        int levels = 0;
        if (ml) {
            std::vector<int64_t> ranking, sizes;
            hierarchy_host(P.n, support_keys(C, P), P.rec_key, P.rec_g, ranking, sizes);
            for (int l = (int)sizes.size() - 1; l >= 0; --l) {
                set_level_keys(C, P, ranking.data(), sizes[l]);
                SweepResult sr = sweep(C, P, false, tolI, tolN);
                blocks += sr.blocks;
                cg_it += sr.cg_iters;
                cd_sw += sr.cd_sweeps;
                ++sweeps;
                ++levels;
            }
        }
        SweepResult sr = sweep(C, P, true, tolI, tolN);
        blocks += sr.blocks;
        cg_it += sr.cg_iters;
        cd_sw += sr.cd_sweeps;
        ++sweeps;
        ++cycles;
        kkt_prev = sr.kkt_max;
        kkt_l1 = sr.kkt_l1;
        if (verbose)
            fprintf(stderr, "[sic] cycle %d levels %d prec %s F=%.15e kkt=%.3e nnz=%lld t=%.3fs\n",
                    cyc, levels, C.prec == PREC_F64 ? "f64" : (C.prec == PREC_F32 ? "f32" : "bf16"),
                    P.F, sr.kkt_max, (long long)P.Acur().nnz, secs());
        if (C.trace && trace_len < C.trace_cap) {
            sic_trace_entry& e = C.trace[trace_len++];
            e.seconds = secs();
            e.objective = P.F;
            e.kkt_max = sr.kkt_max;
            const double l1 = a_l1_norm(C, P);
            e.kkt_rel_l1 = l1 > 0 ? sr.kkt_l1 / l1 : INFINITY;
            e.nnz = P.Acur().nnz;
            e.cycle = cyc;
            e.levels = levels;
        }
        // a reduced-precision cycle measures the KKT with approximate S and W:
        // only a float64 cycle may end the solve, and (unless switched off)
        // only once the exact pass (float64 S_J, W_J by CG to tol_cert)
        // confirms the sweep's measure, which saw each block before its update
        // and W from the sweep's looser CG
        certified = false;
        if (sr.kkt_max <= tol && C.prec == PREC_F64 && P.lam == lam_target) {
            if (!certify) {
                status = SIC_OK;
                break;
            }
            kkt_prev = exact_kkt(C, P, tol_cert, &kkt_l1);
            certified = true;
            if (verbose)
                fprintf(stderr, "[sic] cycle %d exact KKT %.3e (sweep %.3e)\n", cyc, kkt_prev,
                        sr.kkt_max);
            if (kkt_prev <= tol) {
                status = SIC_OK;
                break;
            }
        }
    }
    } catch (const SicError& e) {
        // a conjugate-gradient solve stopped at its iteration cap: the block it
        // served was abandoned before it changed A, so the iterate is the last
        // accepted one (positive definite) and is returned with SIC_ENOCONV
        if (e.code != SIC_ENOCONV) throw;
        if (verbose) fprintf(stderr, "[sic] stopped: %s\n", e.what());
        status = SIC_ENOCONV;
        certified = false;
    }
    C.prec = PREC_F64;
    set_lambda(lam_target);
    double kkt_final = kkt_prev;
    if ((C.opt.flags & SIC_FLAG_FINAL_KKT) && !certified) {
        // the exact measure of whatever iterate the solve ends with
        try {
            kkt_final = exact_kkt(C, P, tol_cert, &kkt_l1);
            status = kkt_final <= tol ? SIC_OK : SIC_ENOCONV;
        } catch (const SicError& e) {
            if (e.code != SIC_ENOCONV) throw;
            status = SIC_ENOCONV;
        }
    }
    if (info) {
        info->objective = P.F;
        info->kkt_max = kkt_final;
        const double l1 = a_l1_norm(C, P);
        info->kkt_rel_l1 = l1 > 0 ? kkt_l1 / l1 : INFINITY;
        info->nnz = P.Acur().nnz;
        info->max_nnz = P.max_nnz;
        info->cycles = cycles;
        info->sweeps = sweeps;
        info->blocks = blocks;
        info->cg_iterations = cg_it;
        info->cd_sweeps = cd_sw;
        info->seconds = secs();
        info->status = status;
        info->trace_len = trace_len;
    }
    return status;
}

// ------------------------------------------------------------------ standalone steps

static void load_coords(Context& C, int jp, int b, const double* wjj, const int64_t* cptr,
                        const int32_t* cp, const double* S, const double* A) {
    BlockWork& W = C.work;
    hipStream_t s = C.stream;
    const int64_t nc = cptr[b];
    const size_t ncs = (size_t)std::max<int64_t>(nc, 1);
    W.WJJ.reserve((size_t)jp * jp);
    W.cptr.reserve(b + 1);
    W.c_p.reserve(ncs); W.c_ci.reserve(ncs); W.c_S.reserve(ncs); W.c_A.reserve(ncs);
    W.c_a.reserve(ncs); W.c_inva.reserve(ncs); W.c_wtc.reserve(ncs); W.c_wtt.reserve(ncs);
    W.delta.reserve(ncs); W.mu.reserve(ncs);
    SIC_HIP(hipMemcpyAsync(W.WJJ.p, wjj, sizeof(double) * jp * jp, hipMemcpyHostToDevice, s));
    SIC_HIP(hipMemcpyAsync(W.cptr.p, cptr, sizeof(int64_t) * (b + 1), hipMemcpyHostToDevice, s));
    if (nc) {
        SIC_HIP(hipMemcpyAsync(W.c_p.p, cp, sizeof(int32_t) * nc, hipMemcpyHostToDevice, s));
        SIC_HIP(hipMemcpyAsync(W.c_S.p, S, sizeof(double) * nc, hipMemcpyHostToDevice, s));
        SIC_HIP(hipMemcpyAsync(W.c_A.p, A, sizeof(double) * nc, hipMemcpyHostToDevice, s));
    }
    launch_cd_prep(W.cptr.p, b, nc, W.c_p.p, W.WJJ.p, jp, W.c_ci.p, W.c_a.p, W.c_inva.p, W.c_wtc.p,
                   W.c_wtt.p, W.delta.p, s);
}

int step_cd_impl(Context& C, int jp, int b, const double* wjj, const int64_t* cptr,
                 const int32_t* cp, const double* S, const double* A, double lambda, int max_sweeps,
                 double tol, double* delta_out, double* stats_out) {
    BlockWork& W = C.work;
    hipStream_t s = C.stream;
    load_coords(C, jp, b, wjj, cptr, cp, S, A);
    const int64_t nc = cptr[b];
    const int64_t cd_rec = run_cd(C, jp, b, nc, lambda, max_sweeps, tol);
    if (nc) SIC_HIP(hipMemcpyAsync(delta_out, W.delta.p, sizeof(double) * nc, hipMemcpyDeviceToHost, s));
    sync(C);
    double st[8];
    std::copy(cd_stats(C), cd_stats(C) + 8, st);
    if (st[7] != 0.0) throw SicError(SIC_EINTERNAL, "CD sweep workgroups timed out waiting on one another");
    prof_scale(cd_rec, st[0]);
    if (stats_out) std::copy(st, st + 7, stats_out);
    return SIC_OK;
}

int step_ls_impl(Context& C, int jp, int b, const double* wjj, const int64_t* cptr,
                 const int32_t* cp, const double* S, const double* A, const double* delta,
                 double lambda, double* alpha, double* dF, int* trials, double* logdet_out,
                 int n_alpha) {
    BlockWork& W = C.work;
    hipStream_t s = C.stream;
    load_coords(C, jp, b, wjj, cptr, cp, S, A);
    const int64_t nc = cptr[b];
    if (nc) SIC_HIP(hipMemcpyAsync(W.delta.p, delta, sizeof(double) * nc, hipMemcpyHostToDevice, s));
    LineSearch ls = line_search(C, lambda, jp, b, jp - b, nc);
    if (!ls.wii_pd) throw SicError(SIC_ENOTPD, "W_II is not positive definite");
    if (alpha) *alpha = ls.alpha;
    if (dF) *dF = ls.dF;
    if (trials) *trials = ls.trials;
    for (int i = 0; logdet_out && i < n_alpha; i += 4) {
        const int nt = std::min(4, n_alpha - i);
        double ld[4], lin[4];
        int pd[4];
        ls_eval(C, b, nc, lambda, i, nt, ld, pd, lin);
        for (int t = 0; t < nt; ++t) logdet_out[i + t] = pd[t] ? ld[t] : NAN;
    }
    return SIC_OK;
}

}  // namespace sic

namespace sic {

int request_results(const sic_problem& q) { return q.n_lambda > 0 ? q.n_lambda : 1; }

int solve_request(Context& C, Problem& P, const sic_problem& q, sic_csr* A_out, sic_info* info) {
    if (!q.X || q.n < 1 || q.m < 1 || !(q.tol > 0.0) || q.n > INT32_MAX ||
        (q.x_dtype != SIC_X_F64 && q.x_dtype != SIC_X_F32 && q.x_dtype != SIC_X_BF16) ||
        (q.n_lambda > 0 && !q.lambda_path))
        throw SicError(SIC_EINVAL, "bad problem");
    const int nl = request_results(q);
    auto lam_at = [&](int l) { return q.n_lambda > 0 ? q.lambda_path[l] : q.lambda; };
    for (int l = 0; l < nl; ++l) {
        const double lam = lam_at(l);
        if (!(lam >= 0.0) || !std::isfinite(lam) || (lam == 0.0 && q.m <= q.n))
            throw SicError(SIC_EINVAL, "bad lambda");
    }
    problem_init(C, P, q.X, q.x_dtype, q.n, q.m, lam_at(0));
    if (q.A0) {
        set_A_host(C, P, q.A0);
        P.F = warm_start_objective(C, P, q.A0);
    }
    int worst = SIC_OK;
    for (int l = 0; l < nl; ++l) {
        const double lam = lam_at(l);
        if (l > 0) {
            // warm start from the previous lambda: F changes by (lam - lam_prev) * ||A||_1
            P.F += (lam - P.lam) * a_l1_norm(C, P);
            P.lam = lam;
        }
        sic_info* inf = info ? &info[l] : nullptr;
        const int st = solve_problem(C, P, q.tol, inf);
        get_A_host(C, P, &A_out[l]);
        if (st != SIC_OK && worst == SIC_OK) worst = st;
    }
    return worst;
}

}  // namespace sic

namespace sic {

void release_workspace(Context& C) {
    sync(C);
    if (C.side) stream_wait(C.side);
    C.work.~BlockWork();
    new (&C.work) BlockWork();
}

}  // namespace sic
