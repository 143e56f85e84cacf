// Host-side state of the solver: context, problem, block working set.
#pragma once

#include "sic_internal.h"

namespace sic {

enum { PREC_F64 = 0, PREC_F32 = 1, PREC_BF16 = 2 };

struct Options {
    int block = 256;
    double cg_tol_I = 1e-5, cg_tol_N = 1e-4;
    int cg_max_iter = 1000;
    double cd_tol = 1e-4;
    int cd_max_sweeps = 20;
    int cd_hessian_max = 4096;   // 0: never use the explicit-Hessian sweep
    int pcd_min_coords = 4097;   // blocks with at least this many coordinates use PCD-CG; 0: never
    int ls_max_trials = 31;
    int max_cycles = 100;
    uint64_t flags = 0;
    int precision = SIC_FP64;
};

// Scratch of one block update; sized on demand, reused across blocks.
struct BlockWork {
    DevBuf<double> SJ, WI, AJ, ANEW, WN, WJJ, U, ug, HT;
    DevBuf<double> cdx;    // exchange buffer of the multi-workgroup CD sweep
    DevBuf<unsigned char> markg;
    DevBuf<char> xstage;   // reduced-precision X before its conversion; relabelled X
    DevBuf<int32_t> perm;  // a relabelling on the device
    DevBuf<int32_t> cols;
    // free lists
    DevBuf<int64_t> colptr;
    DevBuf<int32_t> e_row, tilecount, offsets, nflag, ccount;
    DevBuf<double> e_g, e_s, e_a, e_w, kkt, kkt_acc;
    // neighbourhood
    DevBuf<int64_t> scan_n;
    DevBuf<int32_t> Jp, lmap;
    // coordinates
    DevBuf<int64_t> cptr;
    DevBuf<int32_t> c_p, c_e, c_ci, c_gr, c_gc;
    DevBuf<double> c_S, c_A, c_a, c_inva, c_wtc, c_wtt, delta, mu;
    // line search
    DevBuf<double> Dinv, Rb, D11, Mo, Y, Pm, T1, T2, D1, X, XtX, RPR, E1, E2, C;
    // coarse levels
    DevBuf<int32_t> cand_col, cflag, cmap, NC, err;
    DevBuf<double> S_cand, WNC, WII, Kb, AII;
    // CSR rebuild
    DevBuf<int32_t> rcount;
    // the finest sweep's free pairs and |g| (for the next hierarchy), read back
    // at the block's closing synchronisation
    HostBuf<int64_t> h_cp;
    HostBuf<int32_t> h_rows;
    HostBuf<double> h_g;
    // a second set for the initial free set, whose read-backs alternate
    // between the two while the host records the previous block's pairs
    HostBuf<int64_t> h_cp_alt;
    HostBuf<int32_t> h_rows_alt;
    HostBuf<double> h_g_alt;
    CGWork cg;
    PcdWork pcd;
    int64_t n_init = 0;   // n for which flag/map arrays are initialised
    int b_init = 0;
};

struct BlockResult {
    int64_t j0 = 0;
    int b = 0;
    int level = 0;
    int64_t E = 0, nN = 0, nC = 0, ncoord = 0, jp = 0;
    int cg_iters_I = 0, cg_iters_N = 0;
    double cg_res_I = 0, cg_res_N = 0;
    int cd_sweeps = 0;
    double cd_last_maxmu = 0;
    double alpha = 0, dF = 0;
    int trials = 0;
    int64_t nnz_after = 0;
};

// (the step entry points of sic_steps.h pass warm_allowed = false: their
// conjugate gradients start from zero, as the oracle's do)
constexpr size_t warm_store_max_bytes = (size_t)2 << 30;
inline bool warm_store_fits(int64_t n) { return (double)n * n * 8.0 <= (double)warm_store_max_bytes; }

struct Problem {
    int64_t n = 0, m = 0;
    double lam = 0;
    DevBuf<double> X, Xt, diagS;
    DevBuf<float> Xf;        // narrowed copies of X for the mixed-precision path
    DevBuf<uint16_t> Xb;
    bool narrow = false;
    DevCSR A[2];
    int cur = 0;
    double F = 0;
    int64_t max_nnz = 0;
    // level set C_l as a symmetric CSR pattern (device) plus host row pointers
    DevBuf<int64_t> crow;
    DevBuf<int32_t> ccol;
    std::vector<int64_t> crow_h;
    bool level_set = false;
    // free pairs (key i*n+j, i<=j) and |g| recorded by the last finest sweep
    std::vector<int64_t> rec_key;
    std::vector<double> rec_g;
    std::vector<int64_t> rec_seq;
    // relabelling of the variables (SIC_FLAG_CLUSTER): perm[p] is the caller's
    // label of the variable the solver calls p; empty means none
    std::vector<int32_t> perm;
    // inverse columns as last solved, the conjugate gradients' warm starts:
    // row c of Wst holds column c of A^{-1} when Wvalid[c] (kept when n^2
    // doubles fit in warm_store_max_bytes and SIC_FLAG_NO_WARM_CG is off)
    DevBuf<double> Wst;
    DevBuf<unsigned char> Wvalid;
    bool warm = false;
    // float64 columns of S as formed: row-major n x n, column j valid when
    // s_cached[j] (same size rule; SIC_FLAG_NO_S_CACHE turns it off). S_J of a
    // later cycle is copied out instead of formed again.
    DevBuf<double> Scache;
    std::vector<char> s_cached;
    bool scache = false;
    const WarmStore* warm_store() {
        ws_ = WarmStore{Wst.p, Wvalid.p};
        return warm ? &ws_ : nullptr;
    }
    DevCSR& Acur() { return A[cur]; }
  private:
    WarmStore ws_{nullptr, nullptr};
  public:
};

struct Context {
    int device = 0;
    hipStream_t stream = nullptr;
    // second stream of the context: work of a block update that can run beside
    // the main stream's (forked after, and joined before, events on the main one)
    hipStream_t side = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool own_stream = false;
    Options opt;
    size_t budget = 0;
    std::shared_ptr<MemAccount> acct = std::make_shared<MemAccount>();
    BlockWork work;
    sic_trace_entry* trace = nullptr;
    int trace_cap = 0;
    // pinned staging for small device-to-host reads (64 entries each):
    //   h_i64[0, 4) counts, [8] the rebuilt CSR's entry count, [16] the coarse-level
    //   error flag (int32); h_f64[0, 26) line-search trials, [32] the PCD stop
    //   flag, [40, 48) sweep statistics, [48, 50) the coarse A_II factor's flags.
    //   Most are written by the producing kernels themselves (the memory is
    //   mapped for the device), the rest by copies; either way the host reads
    //   them after waiting for the stream.
    int64_t* h_i64 = nullptr;
    double* h_f64 = nullptr;
    BlockResult last;
    // precision of the current sweep (mixed-precision path): S_J from X in
    // float64, float or bfloat16; CG vectors in float unless PREC_F64
    int prec = PREC_F64;
};

// context set-up (stream, pinned staging, options) and release; the context's
// device workspace is freed with the Context itself
void context_init(Context& C, const sic_options& o);
void context_release(Context& C);
// frees the block workspace (the next block update allocates it again)
void release_workspace(Context& C);

// problem setup / transfer
void problem_init(Context& C, Problem& P, const void* X, int x_dtype, int64_t n, int64_t m,
                  double lam, bool warm_allowed = true);
void set_identity(Context& C, Problem& P);
void set_A_host(Context& C, Problem& P, const sic_csr* A);
void get_A_host(Context& C, Problem& P, sic_csr* out);
void set_level_keys(Context& C, Problem& P, const int64_t* keys, int64_t count);

// algorithm
BlockResult block_update(Context& C, Problem& P, int64_t j0, int b, bool fine, bool record,
                         double tolI, double tolN);
void initial_free_set(Context& C, Problem& P);
struct SweepResult {
    double kkt_max = 0, kkt_l1 = 0;
    int64_t cg_iters = 0, cd_sweeps = 0, blocks = 0;
};
SweepResult sweep(Context& C, Problem& P, bool fine, double tolI, double tolN);
void hierarchy_host(int64_t n, const std::vector<int64_t>& supp,
                    const std::vector<int64_t>& fkey, const std::vector<double>& fg,
                    std::vector<int64_t>& ranking, std::vector<int64_t>& sizes);
std::vector<int64_t> support_keys(Context& C, Problem& P);
// Clustered block partition (cluster.hip): the variables in block order.
std::vector<int32_t> cluster_order(int64_t n, const int64_t* keys, int64_t count, int b);
// Relabels the problem (samples, iterate, recorded free pairs) by the cluster
// order of the graph of A's support and the recorded free pairs.
void cluster_problem(Context& C, Problem& P);
int solve_problem(Context& C, Problem& P, double tol, sic_info* info);
// One request of sic_solve_batch (or of the serving loop): set-up, optional
// warm start, then the lambda path (or the single lambda). Results go to
// A_out[0 .. results) and info[0 .. results); returns the first bad status.
int solve_request(Context& C, Problem& P, const sic_problem& q, sic_csr* A_out, sic_info* info);
int request_results(const sic_problem& q);
double exact_kkt(Context& C, Problem& P, double tol_cg, double* l1);
// F(A0) of a warm start already loaded as the iterate; throws SIC_ENOTPD when
// A0 is not positive definite
double warm_start_objective(Context& C, Problem& P, const sic_csr* A0);

}  // namespace sic
