// Host stand-in for the solver entry points the serving loop calls (test
// infrastructure only): each "solve" allocates through the same accounted
// buffers, reads the caller's samples, sleeps a little and returns a small
// result, so that the serving loop's threads, queue, admission, waits and
// cancellations run for real under the sanitizers.
#include <chrono>
#include <random>
#include <thread>

#include "solver.h"

namespace sic {

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
AccountScope::AccountScope(const std::shared_ptr<MemAccount>& a) : prev_(t_account) { t_account = a; }
AccountScope::~AccountScope() { t_account = prev_; }
void set_blocking_waits(bool) {}

void context_init(Context& C, const sic_options& o) {
    C.device = o.device;
    C.opt.block = o.block > 0 ? o.block : 256;
}
void context_release(Context&) {}
void release_workspace(Context& C) {
    C.work.~BlockWork();
    new (&C.work) BlockWork();
}

int request_results(const sic_problem& q) { return q.n_lambda > 0 ? q.n_lambda : 1; }

int solve_request(Context& C, Problem& P, const sic_problem& q, sic_csr* A_out, sic_info* info) {
    const double* X = static_cast<const double*>(q.X);
    volatile double first = X[0];   // the caller's samples must still be valid
    volatile double last = X[q.n * q.m - 1];
    (void)first;
    (void)last;
    thread_local std::mt19937 rng(std::random_device{}());
    C.work.SJ.reserve((size_t)q.n * 8);
    P.X.reserve((size_t)q.n * q.m);
    std::memcpy(P.X.p, X, sizeof(double) * q.n * q.m);
    std::this_thread::sleep_for(std::chrono::microseconds(200 + rng() % 3000));
    if (q.tol > 0.5) throw SicError(SIC_ENOTPD, "stub failure");
    const int nl = request_results(q);
    for (int l = 0; l < nl; ++l) {
        sic_csr& a = A_out[l];
        a.n = q.n;
        a.nnz = q.n;
        a.rowptr = (int64_t*)malloc(sizeof(int64_t) * (q.n + 1));
        a.col = (int32_t*)malloc(sizeof(int32_t) * q.n);
        a.val = (double*)malloc(sizeof(double) * q.n);
        for (int64_t i = 0; i <= q.n; ++i) a.rowptr[i] = i;
        for (int64_t i = 0; i < q.n; ++i) {
            a.col[i] = (int32_t)i;
            a.val[i] = 1.0 + P.X.p[i];
        }
        if (info) {
            std::memset(&info[l], 0, sizeof(sic_info));
            info[l].nnz = q.n;
            info[l].status = SIC_OK;
        }
    }
    return SIC_OK;
}

}  // namespace sic

extern "C" {
void sic_options_default(sic_options* o) {
    std::memset(o, 0, sizeof(*o));
    o->block = 256;
}
void sic_csr_free(sic_csr* a) {
    if (!a) return;
    free(a->rowptr);
    free(a->col);
    free(a->val);
    std::memset(a, 0, sizeof(*a));
}
}
