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

__device__ inline int64_t lower_bound_col(const int32_t* __restrict__ col, int64_t lo, int64_t hi,
                                          int64_t key) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (col[mid] < key) lo = mid + 1; else hi = mid;
    }
    return lo;
}

// pass 0: count the entries of every new row; pass 1: write them at nrowptr.
__global__ void k_upd_rows(int pass, int64_t n, int64_t j0, int b,
                           const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                           const double* __restrict__ val, const int32_t* __restrict__ lmap,
                           const int64_t* __restrict__ cptr, const int32_t* __restrict__ c_p,
                           const int32_t* __restrict__ Jp, const double* __restrict__ ANEW,
                           int32_t* __restrict__ cnt, const int64_t* __restrict__ nrowptr,
                           int32_t* __restrict__ ncol, double* __restrict__ nval, int64_t cap) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int64_t j1 = j0 + b;
    int64_t o = pass ? nrowptr[r] : 0;
    int64_t count = 0;
    const double* arow = ANEW + r * b;
    auto emit = [&](int64_t c, double v) {
        if (pass) {
            if (o < cap) {   // the host checks the total against cap after the block
                ncol[o] = (int32_t)c;
                nval[o] = v;
            }
            ++o;
        }
        ++count;
    };
    // the dense row over the block columns, 16 loads in flight at a time
    // (unconditional loads of a clamped index, then a select)
    auto emit_dense = [&]() {
        for (int q0 = 0; q0 < b; q0 += 16) {
            double v[16];
#pragma unroll
            for (int u = 0; u < 16; ++u) {
                const int q = q0 + u < b ? q0 + u : b - 1;
                v[u] = arow[q];
            }
#pragma unroll
            for (int u = 0; u < 16; ++u)
                if (q0 + u < b && v[u] != 0.0) emit(j0 + q0 + u, v[u]);
        }
    };
    if (r >= j0 && r < j1) {
        const int ci = (int)(r - j0);
        const int64_t t0 = cptr[ci], t1 = cptr[ci + 1];
        int64_t t = t0;
        for (; t < t1; ++t) {   // coordinates are sorted by row: rows < j0 first
            const int64_t g = Jp[c_p[t]];
            if (g >= j0) break;
            const double v = ANEW[g * b + ci];
            if (v != 0.0) emit(g, v);
        }
        emit_dense();
        for (; t < t1; ++t) {
            const int64_t g = Jp[c_p[t]];
            if (g < j1) continue;
            const double v = ANEW[g * b + ci];
            if (v != 0.0) emit(g, v);
        }
    } else {
        const int64_t e0 = rowptr[r], e1 = rowptr[r + 1];
        const bool in_n = lmap[r] >= b;
        if (!in_n) {
            if (pass) {
                for (int64_t e = e0; e < e1; ++e) emit(col[e], val[e]);
            } else {
                count = e1 - e0;
            }
        } else {
            const int64_t lo = lower_bound_col(col, e0, e1, j0);
            const int64_t hi = lower_bound_col(col, lo, e1, j1);
            for (int64_t e = e0; e < lo; ++e) emit(col[e], val[e]);
            emit_dense();
            for (int64_t e = hi; e < e1; ++e) emit(col[e], val[e]);
        }
    }
    if (!pass) cnt[r] = (int32_t)count;
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
    hipLaunchKernelGGL(k_upd_rows, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, pass, n, j0, b,
                       A.rowptr.p, A.col.p, A.val.p, lmap, cptr, c_p, Jp, ANEW, cnt, nrowptr, ncol,
                       nval, cap);
    SIC_CHECK_LAUNCH();
    prof_end(KK_UPD_ROWS, s, (double)A.nnz * 12.0 * (pass ? 2.0 : 0.0) + (double)n * 16.0, 0.0);
}

}  // namespace sic
