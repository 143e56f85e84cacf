// Inverse columns W_J = A^{-1} E_J by conjugate gradients (Section 6.1: "the
// solution of these linear systems is one of the main computational tasks";
// CG, possibly preconditioned, is the method the paper names). Jacobi
// preconditioner (diag A > 0 for SPD A).
//
// All k right-hand sides run together on row-major n x k blocks, so that one
// sparse row of A gathers whole 64-column segments of the direction block
// (coalesced 512-byte reads) and the per-column CG scalars stay independent.
// One iteration is two kernels:
//   spmm:   p = z + beta p,  q = A z + beta q  (= A p),   partial p.q
//   update: x += alpha p, r -= alpha q, z = D^{-1} r,      partial r.z, r.r
// The per-column reductions finish in the last workgroup to arrive (a fixed
// summation order, so results do not depend on scheduling), which also
// derives alpha, beta and the convergence flag; a converged solve turns the
// remaining queued launches into no-ops.
#include "sic_internal.h"

namespace sic {

namespace {

constexpr int CG_THREADS = 512;     // 8 waves, one matrix row per wave at a time
constexpr int CG_WAVES = CG_THREADS / 64;
constexpr int CG_ROW_TILES = 128;   // row partitions (partials per column)

enum { F_DONE = 0, F_CNT_A = 1, F_CNT_B = 2, F_ITER = 3, F_FIRST = 4 };
enum { S_RZ = 0, S_ALPHA = 1, S_BETA = 2, S_RR = 3 };

__global__ void k_cg_dinv(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                          const double* __restrict__ val, int64_t n, double* __restrict__ dinv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
        if (col[e] == (int32_t)i) d = val[e];
    dinv[i] = d > 0.0 ? 1.0 / d : 1.0;
}

__global__ void k_cg_init(int64_t n, int k, const int32_t* __restrict__ cols,
                          const double* __restrict__ dinv, double* __restrict__ R,
                          double* __restrict__ Z, double* __restrict__ scal,
                          int* __restrict__ flags) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < k) {
        const int64_t c = cols[j];
        R[c * k + j] = 1.0;
        Z[c * k + j] = dinv[c];
        scal[j * 4 + S_RZ] = dinv[c];
        scal[j * 4 + S_ALPHA] = 0.0;
        scal[j * 4 + S_BETA] = 0.0;
        scal[j * 4 + S_RR] = 1.0;
    }
    if (j == 0) {
        flags[F_DONE] = 0;
        flags[F_CNT_A] = 0;
        flags[F_CNT_B] = 0;
        flags[F_ITER] = 0;
        flags[F_FIRST] = 1;
        scal[4 * k] = 1.0;
    }
}

__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

__global__ __launch_bounds__(CG_THREADS) void k_cg_spmm(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, int64_t n, int k, const double* __restrict__ Z,
    double* __restrict__ P, double* __restrict__ Q, double* __restrict__ scal,
    double* __restrict__ part, int* __restrict__ flags) {
    if (__builtin_nontemporal_load(&flags[F_DONE])) return;
    const bool first = flags[F_FIRST] != 0;
    const int lane = threadIdx.x & 63;
    const int wave = wave_id();
    const int j = blockIdx.x * 64 + lane;
    const bool jok = j < k;
    const double beta = (jok && !first) ? scal[j * 4 + S_BETA] : 0.0;
    double pq = 0.0;
    for (int64_t i = (int64_t)blockIdx.y * CG_WAVES + wave; i < n;
         i += (int64_t)gridDim.y * CG_WAVES) {
        const int64_t e0 = rowptr[i], e1 = rowptr[i + 1];
        double acc = 0.0;
        for (int64_t e = e0; e < e1; ++e) {
            const int64_t c = col[e];
            const double a = val[e];
            if (jok) acc += a * Z[c * k + j];
        }
        if (jok) {
            const int64_t o = i * k + j;
            const double z = Z[o];
            const double p = first ? z : z + beta * P[o];
            const double q = first ? acc : acc + beta * Q[o];
            P[o] = p;
            Q[o] = q;
            pq += p * q;
        }
    }
    __shared__ double red[CG_WAVES][64];
    __shared__ int last;
    red[wave][lane] = pq;
    __syncthreads();
    if (wave == 0) {
        double s = 0.0;
        for (int w = 0; w < CG_WAVES; ++w) s += red[w][lane];
        if (jok) part[(int64_t)blockIdx.y * k + j] = s;
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
        last = atomicAdd(&flags[F_CNT_A], 1) == (int)(gridDim.x * gridDim.y) - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    for (int jj = threadIdx.x; jj < k; jj += CG_THREADS) {
        double s = 0.0;
        for (unsigned t = 0; t < gridDim.y; ++t) s += part[(int64_t)t * k + jj];
        const double rz = scal[jj * 4 + S_RZ];
        scal[jj * 4 + S_ALPHA] = (s > 0.0 && rz > 0.0) ? rz / s : 0.0;
    }
    if (threadIdx.x == 0) flags[F_CNT_A] = 0;
}

__global__ __launch_bounds__(CG_THREADS) void k_cg_update(
    int64_t n, int k, const double* __restrict__ dinv, double* __restrict__ W,
    double* __restrict__ R, double* __restrict__ Z, const double* __restrict__ P,
    const double* __restrict__ Q, double* __restrict__ scal, double* __restrict__ part,
    int* __restrict__ flags, double tol) {
    if (__builtin_nontemporal_load(&flags[F_DONE])) return;
    const int lane = threadIdx.x & 63;
    const int wave = wave_id();
    const int j = blockIdx.x * 64 + lane;
    const bool jok = j < k;
    const double alpha = jok ? scal[j * 4 + S_ALPHA] : 0.0;
    double rz = 0.0, rr = 0.0;
    if (jok) {
        for (int64_t i = (int64_t)blockIdx.y * CG_WAVES + wave; i < n;
             i += (int64_t)gridDim.y * CG_WAVES) {
            const int64_t o = i * k + j;
            W[o] += alpha * P[o];
            const double r = R[o] - alpha * Q[o];
            R[o] = r;
            const double z = dinv[i] * r;
            Z[o] = z;
            rz += r * z;
            rr += r * r;
        }
    }
    __shared__ double red[2][CG_WAVES][64];
    __shared__ int last;
    __shared__ double wmax[CG_WAVES];
    red[0][wave][lane] = rz;
    red[1][wave][lane] = rr;
    __syncthreads();
    if (wave == 0) {
        double s0 = 0.0, s1 = 0.0;
        for (int w = 0; w < CG_WAVES; ++w) {
            s0 += red[0][w][lane];
            s1 += red[1][w][lane];
        }
        if (jok) {
            part[((int64_t)blockIdx.y * k + j) * 2 + 0] = s0;
            part[((int64_t)blockIdx.y * k + j) * 2 + 1] = s1;
        }
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0)
        last = atomicAdd(&flags[F_CNT_B], 1) == (int)(gridDim.x * gridDim.y) - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    double mx = 0.0;
    for (int jj = threadIdx.x; jj < k; jj += CG_THREADS) {
        double s0 = 0.0, s1 = 0.0;
        for (unsigned t = 0; t < gridDim.y; ++t) {
            s0 += part[((int64_t)t * k + jj) * 2 + 0];
            s1 += part[((int64_t)t * k + jj) * 2 + 1];
        }
        const double rz_old = scal[jj * 4 + S_RZ];
        scal[jj * 4 + S_BETA] = rz_old > 0.0 ? s0 / rz_old : 0.0;
        scal[jj * 4 + S_RZ] = s0;
        scal[jj * 4 + S_RR] = s1;
        mx = fmax(mx, sqrt(s1));
    }
    for (int off = 32; off > 0; off >>= 1) mx = fmax(mx, __shfl_xor(mx, off, 64));
    if (lane == 0) wmax[wave] = mx;
    __syncthreads();
    if (threadIdx.x == 0) {
        double m = 0.0;
        for (int w = 0; w < CG_WAVES; ++w) m = fmax(m, wmax[w]);
        scal[4 * k] = m;
        flags[F_ITER] += 1;
        flags[F_FIRST] = 0;
        flags[F_CNT_B] = 0;
        if (m <= tol) flags[F_DONE] = 1;
    }
}

}  // namespace

CGResult block_cg(const DevCSR& A, const int32_t* d_cols, int k, double* W, int64_t ldw,
                  double tol, int max_iter, CGWork& wk, hipStream_t s) {
    CGResult res;
    const int64_t n = A.n;
    if (k <= 0) {
        res.converged = true;
        return res;
    }
    if (ldw != k) throw SicError(SIC_EINTERNAL, "block_cg expects ldw == k");
    const size_t nk = (size_t)n * (size_t)k;
    wk.R.reserve(nk);
    wk.Z.reserve(nk);
    wk.P.reserve(nk);
    wk.Q.reserve(nk);
    wk.dinv.reserve(n);
    const int col_tiles = (k + 63) / 64;
    int row_tiles = (int)std::min<int64_t>(CG_ROW_TILES, (n + CG_WAVES - 1) / CG_WAVES);
    if (row_tiles < 1) row_tiles = 1;
    wk.part.reserve((size_t)row_tiles * k * 2);
    wk.scal.reserve((size_t)4 * k + 1);
    wk.flags.reserve(8);
    SIC_HIP(hipMemsetAsync(W, 0, nk * sizeof(double), s));
    SIC_HIP(hipMemsetAsync(wk.R.p, 0, nk * sizeof(double), s));
    SIC_HIP(hipMemsetAsync(wk.Z.p, 0, nk * sizeof(double), s));
    hipLaunchKernelGGL(k_cg_dinv, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       A.rowptr.p, A.col.p, A.val.p, n, wk.dinv.p);
    SIC_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_cg_init, dim3((unsigned)((k + 255) / 256)), dim3(256), 0, s, n, k, d_cols,
                       wk.dinv.p, wk.R.p, wk.Z.p, wk.scal.p, wk.flags.p);
    SIC_CHECK_LAUNCH();
    dim3 grid(col_tiles, row_tiles);
    int host_flags[8];
    double host_res = 0.0;
    int launched = 0;
    while (launched < max_iter) {
        const int chunk = std::min(launched < 16 ? 4 : 8, max_iter - launched);
        for (int c = 0; c < chunk; ++c) {
            hipLaunchKernelGGL(k_cg_spmm, grid, dim3(CG_THREADS), 0, s, A.rowptr.p, A.col.p,
                               A.val.p, n, k, wk.Z.p, wk.P.p, wk.Q.p, wk.scal.p, wk.part.p,
                               wk.flags.p);
            SIC_CHECK_LAUNCH();
            hipLaunchKernelGGL(k_cg_update, grid, dim3(CG_THREADS), 0, s, n, k, wk.dinv.p, W,
                               wk.R.p, wk.Z.p, wk.P.p, wk.Q.p, wk.scal.p, wk.part.p, wk.flags.p,
                               tol);
            SIC_CHECK_LAUNCH();
        }
        launched += chunk;
        SIC_HIP(hipMemcpyAsync(host_flags, wk.flags.p, 5 * sizeof(int), hipMemcpyDeviceToHost, s));
        SIC_HIP(hipMemcpyAsync(&host_res, wk.scal.p + 4 * k, sizeof(double), hipMemcpyDeviceToHost, s));
        SIC_HIP(hipStreamSynchronize(s));
        if (host_flags[F_DONE]) break;
    }
    res.iterations = host_flags[F_ITER];
    res.converged = host_flags[F_DONE] != 0;
    res.max_rel_res = host_res;
    return res;
}

}  // namespace sic
