// Internal declarations of the sic library (not part of the public C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstdint>
#include <cstdio>
#include <memory>
#include <stdexcept>
#include <string>
#include <vector>

#include "sic.h"

namespace sic {

struct HipError : std::runtime_error {
    hipError_t code;
    HipError(hipError_t c, const std::string& what) : std::runtime_error(what), code(c) {}
};

struct SicError : std::runtime_error {
    int code;
    SicError(int c, const std::string& what) : std::runtime_error(what), code(c) {}
};

#define SIC_HIP(expr)                                                                          \
    do {                                                                                       \
        hipError_t _e = (expr);                                                                \
        if (_e != hipSuccess)                                                                  \
            throw ::sic::HipError(_e, std::string(#expr) + ": " + hipGetErrorString(_e));     \
    } while (0)

#define SIC_CHECK_LAUNCH() SIC_HIP(hipGetLastError())

// Device bytes held by one owner (a context or a serving slot), with an
// optional cap. Every DevBuf charges the account that was current on its
// thread when it allocated, and keeps it alive until it frees.
struct MemAccount {
    std::atomic<size_t> bytes{0};
    std::atomic<size_t> budget{0};   // 0: no cap
};
// The account of the calling thread (a process-wide uncapped one by default).
const std::shared_ptr<MemAccount>& current_account();
// Makes `a` the calling thread's account for the lifetime of the scope.
struct AccountScope {
    explicit AccountScope(const std::shared_ptr<MemAccount>& a);
    ~AccountScope();
    AccountScope(const AccountScope&) = delete;
    AccountScope& operator=(const AccountScope&) = delete;
  private:
    std::shared_ptr<MemAccount> prev_;
};
// Waits for everything queued on stream s (of the current device) so far:
// polls an event for up to two milliseconds (the host sees completion within
// microseconds, where a blocking wait can sleep through tens of them), then
// blocks. The solver's read-backs, all on the critical path, wait this way.
void stream_wait(hipStream_t s);
// Makes the calling thread's stream waits block without polling (the serving
// workers, which would otherwise spin side by side).
void set_blocking_waits(bool on);

// Largest dynamic LDS a workgroup may use on the current device.
extern size_t CD_MAX_LDS_BYTES;

// Device buffer with grow-only capacity (contents are not kept on growth).
template <typename T>
struct DevBuf {
    T* p = nullptr;
    size_t cap = 0;
    std::shared_ptr<MemAccount> acct;
    DevBuf() = default;
    DevBuf(const DevBuf&) = delete;
    DevBuf& operator=(const DevBuf&) = delete;
    ~DevBuf() { release(); }
    void release() {
        if (p) {
            (void)hipFree(p);
            acct->bytes -= cap * sizeof(T);
        }
        p = nullptr;
        cap = 0;
        acct.reset();
    }
    void reserve(size_t count) {
        if (count <= cap && p) return;
        release();
        size_t bytes = (count ? count : 1) * sizeof(T);
        const std::shared_ptr<MemAccount>& a = current_account();
        const size_t cap_bytes = a->budget.load();
        if (cap_bytes && a->bytes.load() + bytes > cap_bytes)
            throw SicError(SIC_ENOMEM, "HBM budget exceeded by a " + std::to_string(bytes) +
                                           "-byte buffer");
        hipError_t e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            throw SicError(SIC_ENOMEM, "device allocation of " + std::to_string(bytes) + " bytes failed");
        }
        cap = count ? count : 1;
        acct = a;
        acct->bytes += cap * sizeof(T);
    }
    // reserve for a size that creeps up over calls: grows by at least half the
    // capacity, so a slowly growing count reallocates (and synchronises the
    // device in hipFree) a logarithmic number of times
    void reserve_grow(size_t count) {
        if (count <= cap && p) return;
        reserve(std::max(count, cap + cap / 2));
    }
};

// Pinned host buffer with grow-only capacity, for read-backs the host waits on
// (a copy into pageable memory goes through a staging buffer and its own wait).
template <typename T>
struct HostBuf {
    T* p = nullptr;
    size_t cap = 0;
    HostBuf() = default;
    HostBuf(const HostBuf&) = delete;
    HostBuf& operator=(const HostBuf&) = delete;
    ~HostBuf() {
        if (p) (void)hipHostFree(p);
    }
    void reserve(size_t count) {
        if (count <= cap && p) return;
        if (p) (void)hipHostFree(p);
        p = nullptr;
        cap = 0;
        const size_t c = count ? count : 1;
        if (hipHostMalloc((void**)&p, c * sizeof(T), hipHostMallocDefault) != hipSuccess) {
            p = nullptr;
            (void)hipGetLastError();
            throw SicError(SIC_ENOMEM, "pinned host allocation failed");
        }
        cap = c;
    }
    // grows by at least half the capacity (pinned allocations are slow)
    void reserve_grow(size_t count) {
        if (count <= cap && p) return;
        reserve(std::max(count, cap + cap / 2));
    }
};

// Symmetric sparse matrix on the device: full CSR (both triangles), sorted columns.
struct DevCSR {
    int64_t n = 0, nnz = 0;
    DevBuf<int64_t> rowptr;
    DevBuf<int32_t> col;
    DevBuf<double> val;
};

// ---------------------------------------------------------------- k_sj.hip
void launch_sj_gemm_f64(const double* X, int64_t n, int64_t m, int64_t j0, int b, double* out,
                        hipStream_t s);
// S_J from a float or bfloat16 copy of X (float accumulation, float64 result)
void launch_sj_gemm_low(const void* X, bool bf16, int64_t n, int64_t m, int64_t j0, int b,
                        double* out, hipStream_t s);
// narrowed copies of X (either output may be null)
void launch_narrow(const double* X, int64_t count, float* xf, uint16_t* xb, hipStream_t s);
void launch_transpose(const double* X, int64_t m, int64_t n, double* Xt, hipStream_t s);
void launch_diag_s(const double* Xt, int64_t n, int64_t m, double* d, hipStream_t s);
void launch_sddmm(const double* Xt, int64_t m, const int32_t* rows, const int32_t* cols,
                  int64_t count, double* out, hipStream_t s);

// ---------------------------------------------------------------- k_cg.hip
struct CGWork {
    DevBuf<double> R, P, Q, dinv, vd, part, scal;
    DevBuf<float> R32, P32, Q32;        // the float vectors of the reduced-precision CG
    DevBuf<int32_t> flags;
    HostBuf<int32_t> hctl;              // per-tile control words, read back at each check
    HostBuf<double> hres;               // per-tile relative residuals
    // iterations of the last solve of each kind (caller's slot x precision): the
    // first convergence check comes when a solve like it would have converged
    int predict[8] = {0, 0, 0, 0, 0, 0, 0, 0};
};
struct CGResult {
    int iterations = 0;
    double max_rel_res = 0;
    bool converged = false;   // every column reached tol within max_iter
    bool breakdown = false;   // some direction had p.Ap <= 0: A is not positive definite
};
// A CG solve that broke down (SIC_ENOTPD) or stopped at its iteration cap
// (SIC_ENOCONV) leaves W inexact; this throws, so that no step uses it.
void check_cg(const CGResult& r, const char* what);
// low_precision: float vectors with float64 iterate, scalars and sums, and the
// true residual recomputed in float64 every few iterations (tol >= ~1e-6).
// slot (0..3) names the caller's kind of solve for the iteration prediction.
// A store of inverse columns for warm starts: row c of W (n x n row-major)
// holds column c of A^{-1} as last solved, when valid[c] != 0.
struct WarmStore {
    double* W;
    unsigned char* valid;
};
// ws (may be null): start every column from the store (x0 = 0 where it holds
// none) and write the converged columns back into it.
CGResult block_cg(const DevCSR& A, const int32_t* d_cols, int k, double* W, int64_t ldw,
                  double tol, int max_iter, CGWork& wk, hipStream_t s,
                  bool low_precision = false, int slot = 0, const WarmStore* ws = nullptr);

// The same solve with every buffer in a static per-device array: no device
// or host allocation. All pointers are device pointers. Throws SIC_ETOOBIG
// when the solve does not fit (cg_noalloc_bytes > cg_noalloc_capacity, or
// k > cg_noalloc_max_k). Calls that overlap on one device share the array.
CGResult block_cg_noalloc(const int64_t* rowptr, const int32_t* col, const double* val,
                          int64_t n, int64_t nnz, const int32_t* d_cols, int k, double* W,
                          double tol, int max_iter, hipStream_t s);
size_t cg_noalloc_bytes(int64_t n, int64_t nnz, int k);
size_t cg_noalloc_capacity();
int cg_noalloc_max_k();

// ---------------------------------------------------------------- k_util.hip
void launch_scan_i32(const int32_t* in, int64_t count, int64_t* out, int64_t* total, hipStream_t s);
// total (may be null, or pinned host memory): colptr[b] written there as well
void launch_scan_colmajor(const int32_t* cnt, int tiles, int b, int32_t* offsets, int64_t* colptr,
                          int64_t* total, hipStream_t s);
void launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s);
void launch_iota_i32(int32_t* p, int64_t count, int32_t start, hipStream_t s);
// out (m x n row-major) = the columns perm[0..n) of X (m x n row-major)
void launch_gather_cols(const double* X, int64_t m, int64_t n, const int32_t* perm, double* out,
                        hipStream_t s);
// global (row, column) of every coordinate: Jp[c_p[t]], j0 + c_ci[t]
void launch_coord_globals(int64_t nc, const int32_t* c_p, const int32_t* c_ci, const int32_t* Jp,
                          int64_t j0, int32_t* gr, int32_t* gc, hipStream_t s);

// ---------------------------------------------------------------- k_screen.hip
void launch_scatter_aj(const DevCSR& A, int64_t j0, int b, double* AJ, hipStream_t s);
void launch_screen_fine(int pass, int64_t n, int64_t j0, int b, int rows_per_tile, int tiles,
                        double lam, const double* SJ, const double* WI, const double* AJ,
                        int32_t* tilecount, const int32_t* offsets, int32_t* e_row, double* e_g,
                        double* e_s, double* e_a, double* e_w, int32_t* nflag, double* kkt,
                        hipStream_t s);
void launch_kkt_accumulate(const double* kkt, int tiles, double* acc, hipStream_t s);
void launch_nbr_compact(const int32_t* flag, const int64_t* scan, int64_t n, int64_t j0, int b,
                        int32_t* Jp, int32_t* lmap, hipStream_t s);
void launch_flag_compact(const int32_t* flag, const int64_t* scan, int64_t n, int32_t* list,
                         int32_t* map, hipStream_t s);
void launch_reset_rows(const int32_t* list, int64_t count, int32_t* flag, int32_t* map, hipStream_t s);
void launch_coord_count(const int64_t* colptr, const int32_t* e_row, int64_t j0, int b,
                        int32_t* ccount, hipStream_t s);
void launch_coord_fill(const int64_t* colptr, const int32_t* e_row, const double* e_s,
                       const double* e_a, const int64_t* cptr, const int32_t* lmap, int64_t j0,
                       int b, int32_t* c_p, int32_t* c_e, double* c_S, double* c_A, hipStream_t s);
void launch_gather_wjj(int mode, const int32_t* Jp, int jp, int b, const double* WI,
                       const double* WN, int64_t nN, const double* WII, const double* WNC,
                       int64_t nC, const int32_t* cmap, double* WJJ, hipStream_t s);
void launch_expand_cand(const int64_t* crow, int64_t j0, int b, int64_t base, int32_t* cand_col,
                        hipStream_t s);
void launch_flag_cand(const int32_t* ccol, int64_t base, int64_t count, int64_t j0, int b,
                      int32_t* flag, hipStream_t s);
void launch_a2_k(const DevCSR& A, int64_t j0, int b, const double* WNC, int64_t nC,
                 const int32_t* cmap, double* K, int32_t* err, hipStream_t s);
void launch_dense_aii(const DevCSR& A, int64_t j0, int b, double* out, hipStream_t s);
void launch_screen_coarse(int pass, const int64_t* crow, const int32_t* ccol, int64_t base,
                          int64_t j0, int b, double lam, const double* S_cand, const double* WII,
                          const double* WNC, int64_t nC, const int32_t* cmap, const double* AJ,
                          int32_t* ccount, const int64_t* colptr, int32_t* e_row, double* e_g,
                          double* e_s, double* e_a, double* e_w, int32_t* nflag, hipStream_t s);

// ---------------------------------------------------------------- k_cd.hip
size_t cd_lds_bytes(int jp, bool u_in_lds);
void launch_cd_prep(const int64_t* cptr, int b, int64_t ncoord, const int32_t* c_p,
                    const double* WJJ, int jp, int32_t* c_ci, double* c_a, double* c_inva,
                    double* c_wtc, double* c_wtt, double* delta, hipStream_t s);
void launch_cd(int jp, int b, const int64_t* cptr, const int32_t* c_p, const double* c_S,
               const double* c_A, const double* c_inva, const double* c_wtc, const double* WJJ,
               double lam, int max_sweeps, double tol, double* U, double* delta, double* mu_col,
               double* ug, unsigned char* markg, double* stats, hipStream_t s);
// Explicit coordinate Hessian form: builds H^T (ncoord^2 doubles at HT), then
// runs the sweeps; requires cd_hessian_lds_bytes(ncoord) <= CD_MAX_LDS_BYTES.
// low: H stored as float (in the first half of HT) when the multi-workgroup sweep
// runs, the sweep's arithmetic still float64 (the reduced-precision cycles).
int64_t cd_hessian_limit();   // largest coordinate count the explicit-Hessian sweep takes
size_t cd_hessian_lds_bytes(int64_t ncoord);
// Returns the profiler record of the sweep kernel (bytes and flops of one sweep),
// to be scaled by the sweep count, or -1.
int64_t launch_cd_hessian(int64_t ncoord, int jp, const int32_t* c_p, const int32_t* c_ci,
                          const double* WJJ, const double* c_S, const double* c_A,
                          const double* c_inva, const double* c_wtc, double lam, int max_sweeps,
                          double tol, double* HT, double* delta, double* stats, double* xbuf,
                          hipStream_t s, bool low = false);
// Doubles of the exchange buffer (xbuf above) through which the workgroups of
// the multi-workgroup sweep pass step lists and partial gradients; with a null
// xbuf the sweep runs on one workgroup. stats[7] != 0 after the sweep: its
// workgroups gave up waiting on one another (the result is not usable).
size_t cd_exchange_doubles();

// ---------------------------------------------------------------- k_pcd.hip
struct PcdWork {
    DevBuf<double> z, Y, pdiag, part, sc;
    DevBuf<double> d[2], p[2], zp[2];
    DevBuf<int32_t> dg;
};
// Newton direction by PCD-CG on the free coordinates (delta: in, zero; out,
// the direction). Returns the profiler record (bytes and flops of one
// iteration, to be scaled by the iteration count in stats[0]) or -1. Reads the
// stop flag through the pinned double h_flag every four iterations.
int64_t launch_pcd(int64_t nc, int jp, int b, const int64_t* cptr, const int32_t* c_p,
                   const int32_t* c_ci, const double* c_S, const double* c_A,
                   const double* c_wtc, const double* c_inva, const double* WJJ, double lam,
                   int max_iter, double tol, double* delta, PcdWork& wk, double* stats,
                   double* h_flag, hipStream_t s);

// ---------------------------------------------------------------- k_dense.hip
// dinv (batch 1 only, may be null) receives the inverses of the factor's
// 16 x 16 diagonal blocks (16 x 256 doubles), which launch_trsm_lower consumes.
void launch_chol(double* M, int64_t stride, int batch, int nb, int ld, int identity, double* out,
                 hipStream_t s, double* dinv = nullptr);
void launch_zero_upper(double* M, int nb, int ld, hipStream_t s);
// dense n x n row-major copy of a full symmetric CSR
void launch_csr_to_dense(const int64_t* rowptr, const int32_t* col, const double* val, int64_t n,
                         double* D, hipStream_t s);
void launch_trsm_lower(const double* L, int nb, int ldl, const double* dinv, double* B, int ncols,
                       int ldb, int trans, hipStream_t s);
void launch_gemm_small(int M, int N, int K, double alpha, const double* A, int lda, int ta,
                       const double* B, int ldb, int tb, double beta, double* C, int ldc,
                       hipStream_t s);
void launch_copy_block(const double* src, int ld, int nb, double* dst, hipStream_t s);
void launch_ls_terms(const int64_t* cptr, const int32_t* c_p, const double* delta,
                     const double* WJJ, int jp, int b, int nN, double* D11, double* Mo, double* Y,
                     double* P, hipStream_t s);
void launch_ls_e(const double* D1, const double* X, const double* XtX, const double* RPR, int b,
                 double* E1, double* E2, hipStream_t s);
// Trial steps alpha = 2^-(first + t), t < ntrial (formed on the device).
void launch_ls_trials(const double* E1, const double* E2, int b, int first, int ntrial,
                      double* C, hipStream_t s);
void launch_ls_linear(int64_t ncoord, const int32_t* c_p, const int32_t* c_ci, const double* c_S,
                      const double* c_A, const double* delta, double lam, int first,
                      int ntrial, double* lin, hipStream_t s);
void launch_identity_minus(const double* K, int b, double* out, hipStream_t s);

// ---------------------------------------------------------------- k_update.hip
void launch_upd_newvals(int64_t ncoord, const int32_t* c_p, const int32_t* c_ci, const double* c_A,
                        const double* delta, double alpha, const int32_t* Jp, int64_t j0, int b,
                        double* ANEW, hipStream_t s);
void launch_upd_reset(int64_t ncoord, const int32_t* c_p, const int32_t* c_ci, const int32_t* Jp,
                      int64_t j0, int b, double* ANEW, hipStream_t s);
void launch_upd_rows(int pass, int64_t n, int64_t j0, int b, const DevCSR& A, const int32_t* lmap,
                     const int64_t* cptr, const int32_t* c_p, const int32_t* Jp, const double* ANEW,
                     int32_t* cnt, const int64_t* nrowptr, int32_t* ncol, double* nval,
                     hipStream_t s, int64_t cap = 0);   // pass 1 writes only below cap

}  // namespace sic
