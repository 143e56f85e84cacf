// A <- A + alpha * Delta for one block (Algorithm 2, last step), rebuilding
// the symmetric CSR whose structure changes (entries enter and, when a value
// becomes exactly zero, leave the support).
//
// Every changed entry comes from a descent coordinate (r, c), c in I, which
// decides the unordered pair once, so the result is symmetric by construction.
// The new values of the block are first written into a dense n x b scratch
// (row r, block column c) together with their in-block mirrors; then
//   rows r in I    = out-of-block coordinates of column r (rows < j0),
//                    the dense row r over the block columns, then the
//                    out-of-block coordinates with rows >= j0 + b;
//   rows r in N    = old entries left of the block, the dense row r, old
//                    entries right of the block;
//   all other rows are copied (they have no entry in the block columns).
#include "profiler.h"

namespace sic {

namespace {

__device__ inline double new_value(double a, double alpha, double d) {
    const double s = alpha * d;
    return s == 0.0 ? a : a + s;
}

__global__ void k_upd_newvals(int64_t ncoord, const int32_t* __restrict__ c_p,
                              const int32_t* __restrict__ c_ci, const double* __restrict__ c_A,
                              const double* __restrict__ delta, double alpha,
                              const int32_t* __restrict__ Jp, int64_t j0, int b,
                              double* __restrict__ ANEW) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncoord) return;
    const int p = c_p[t], ci = c_ci[t];
    const int64_t r = Jp[p];
    const double v = new_value(c_A[t], alpha, delta[t]);
    ANEW[r * b + ci] = v;
    if (p < b) ANEW[(j0 + ci) * b + p] = v;
}

__global__ void k_upd_reset(int64_t ncoord, const int32_t* __restrict__ c_p,
                            const int32_t* __restrict__ c_ci, const int32_t* __restrict__ Jp,
                            int64_t j0, int b, double* __restrict__ ANEW) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncoord) return;
    const int p = c_p[t], ci = c_ci[t];
    const int64_t r = Jp[p];
    ANEW[r * b + ci] = 0.0;
    if (p < b) ANEW[(j0 + ci) * b + p] = 0.0;
}

// pass 0: count the entries of every new row; pass 1: write them at nrowptr.
// One wavefront per row: the lanes walk a row's entries 64 at a time and the
// kept ones are compacted in order with a ballot, so a row's dense part over
// the block columns costs b/64 coalesced loads rather than b serial ones.
constexpr int UPD_ROWS_PER_WG = 4;

__global__ __launch_bounds__(64 * UPD_ROWS_PER_WG) void k_upd_rows(
    int pass, int64_t n, int64_t j0, int b, const int64_t* __restrict__ rowptr,
    const int32_t* __restrict__ col, const double* __restrict__ val,
    const int32_t* __restrict__ lmap, const int64_t* __restrict__ cptr,
    const int32_t* __restrict__ c_p, const int32_t* __restrict__ Jp,
    const double* __restrict__ ANEW, int32_t* __restrict__ cnt,
    const int64_t* __restrict__ nrowptr, int32_t* __restrict__ ncol,
    double* __restrict__ nval, int64_t cap) {
    const int lane = threadIdx.x & 63;
    const int64_t r = (int64_t)blockIdx.x * UPD_ROWS_PER_WG + (threadIdx.x >> 6);
    if (r >= n) return;   // whole wavefronts leave together
    const unsigned long long below = (1ull << lane) - 1ull;
    const int64_t j1 = j0 + b;
    const int64_t o0 = pass ? nrowptr[r] : 0;
    int64_t o = o0;
    // keep (c, v) on the lanes where `keep` holds, in lane order after what is there
    auto put = [&](bool keep, int64_t c, double v) {
        const unsigned long long m = __ballot(keep);
        if (pass && keep) {
            const int64_t p = o + __popcll(m & below);
            if (p < cap) {   // the host checks the total against cap after the block
                ncol[p] = (int32_t)c;
                nval[p] = v;
            }
        }
        o += __popcll(m);
    };
    const double* arow = ANEW + r * b;
    auto put_dense = [&]() {
        for (int q0 = 0; q0 < b; q0 += 64) {
            const int q = q0 + lane;
            const double v = arow[q < b ? q : b - 1];
            put(q < b && v != 0.0, j0 + q, v);
        }
    };
    if (r >= j0 && r < j1) {
        // out-of-block coordinates of column r, sorted by row: rows < j0, the
        // dense row, then rows >= j1 (in-block rows are in the dense row)
        const int ci = (int)(r - j0);
        const int64_t t0 = cptr[ci], t1 = cptr[ci + 1];
        for (int side = 0; side < 2; ++side) {
            if (side == 1) put_dense();
            for (int64_t u = t0; u < t1; u += 64) {
                const int64_t t = u + lane;
                const bool in = t < t1;
                const int64_t g = Jp[c_p[in ? t : t0]];
                const double v = ANEW[g * b + ci];
                put(in && (side ? g >= j1 : g < j0) && v != 0.0, g, v);
            }
        }
    } else {
        const int64_t e0 = rowptr[r], e1 = rowptr[r + 1];
        if (lmap[r] < b) {   // not in N: the row has no entry in the block columns
            if (pass) {
                for (int64_t u = e0; u < e1; u += 64) {
                    const int64_t e = u + lane;
                    const bool in = e < e1;
                    const int64_t ee = in ? e : e0;
                    put(in, col[ee], val[ee]);
                }
            } else {
                o = e1 - e0;
            }
        } else {
            // old entries left of the block, the dense row, old entries right of it
            for (int side = 0; side < 2; ++side) {
                if (side == 1) put_dense();
                for (int64_t u = e0; u < e1; u += 64) {
                    const int64_t e = u + lane;
                    const bool in = e < e1;
                    const int64_t ee = in ? e : e0;
                    const int64_t c = col[ee];
                    put(in && (side ? c >= j1 : c < j0), c, val[ee]);
                }
            }
        }
    }
    if (!pass && lane == 0) cnt[r] = (int32_t)(o - o0);
}

}  // namespace

void launch_upd_newvals(int64_t ncoord, const int32_t* c_p, const int32_t* c_ci, const double* c_A,
                        const double* delta, double alpha, const int32_t* Jp, int64_t j0, int b,
                        double* ANEW, hipStream_t s) {
    if (ncoord <= 0) return;
    hipLaunchKernelGGL(k_upd_newvals, dim3((unsigned)((ncoord + 255) / 256)), dim3(256), 0, s,
                       ncoord, c_p, c_ci, c_A, delta, alpha, Jp, j0, b, ANEW);
    SIC_CHECK_LAUNCH();
}

void launch_upd_reset(int64_t ncoord, const int32_t* c_p, const int32_t* c_ci, const int32_t* Jp,
                      int64_t j0, int b, double* ANEW, hipStream_t s) {
    if (ncoord <= 0) return;
    hipLaunchKernelGGL(k_upd_reset, dim3((unsigned)((ncoord + 255) / 256)), dim3(256), 0, s, ncoord,
                       c_p, c_ci, Jp, j0, b, ANEW);
    SIC_CHECK_LAUNCH();
}

void launch_upd_rows(int pass, int64_t n, int64_t j0, int b, const DevCSR& A, const int32_t* lmap,
                     const int64_t* cptr, const int32_t* c_p, const int32_t* Jp, const double* ANEW,
                     int32_t* cnt, const int64_t* nrowptr, int32_t* ncol, double* nval,
                     hipStream_t s, int64_t cap) {
    prof_begin(KK_UPD_ROWS, s);
    hipLaunchKernelGGL(k_upd_rows, dim3((unsigned)((n + UPD_ROWS_PER_WG - 1) / UPD_ROWS_PER_WG)),
                       dim3(64 * UPD_ROWS_PER_WG), 0, s, pass, n, j0, b,
                       A.rowptr.p, A.col.p, A.val.p, lmap, cptr, c_p, Jp, ANEW, cnt, nrowptr, ncol,
                       nval, cap);
    SIC_CHECK_LAUNCH();
    prof_end(KK_UPD_ROWS, s, (double)A.nnz * 12.0 * (pass ? 2.0 : 0.0) + (double)n * 16.0, 0.0);
}

}  // namespace sic
