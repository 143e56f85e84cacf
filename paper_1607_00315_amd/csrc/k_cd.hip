// Newton direction of one block by cyclic coordinate descent on the quadratic
// model (Section 5.1 eq. (Quad_MLE_l1_prior), restricted to the block free set
// of Section 6.1 eq. (active_set_j)).
//
// For the symmetric pair (r, c) the model along Delta_rc = Delta_cr is the 1-D
// problem 0.5*a*mu^2 + b*mu + lam*|x + mu| (Section 3.2, eq. (1d_l1)) with
//   a = W_rc^2 + W_rr W_cc   (W_cc^2 on the diagonal)
//   b = S_rc - W_rc + (W Delta W)_rc,   x = A_rc + Delta_rc
//   mu = -x + soft(x - b/a, lam/a).
// The Hessian term (W Delta W)_rc = sum_p W_rp U_pc uses U = Delta W_{J', I}
// (Section 6.1.1: only the block columns of W Delta W are needed and only
// |J'| rows of W). Coordinates are visited column by column (the order the
// free set is stored in); inside one column only U_rc and U_cc change, so:
//   1. u = U[:, c] is staged in LDS,
//   2. the dots z_k = W_{r_k, J'} u for every coordinate of the column run in
//      parallel across the workgroup (wave reductions),
//   3. one wave walks the column's coordinates in order; after each step it
//      updates every later z_k in its own lane with the rank-2 correction
//      mu * (W_{r_k r} W_cc + W_{r_k c} W_rc), so the serial chain is a few
//      scalar FP64 operations long instead of a length-|J'| dot product,
//   4. the column's steps are folded into U (two row updates each) before
//      the next column.
// One workgroup per block: the chain is inherently sequential; everything
// around it is spread over 8 waves.
#include "sic_internal.h"

namespace sic {

namespace {

constexpr int CD_THREADS = 512;
constexpr int CD_WAVES = CD_THREADS / 64;
constexpr int CD_CHUNK = 64;
constexpr int CD_WPAD = CD_CHUNK + 1;

__device__ inline double readlane_d(double v, int l) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__device__ inline double wave_max(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Per-coordinate constants: the column, a, 1/a, W_rc, W_rr, and zero Delta.
__global__ void k_cd_prep(const int64_t* __restrict__ cptr, int b, int64_t ncoord,
                          const int32_t* __restrict__ c_p, const double* __restrict__ WJJ, int jp,
                          int32_t* __restrict__ c_ci, double* __restrict__ c_a,
                          double* __restrict__ c_inva, double* __restrict__ c_wtc,
                          double* __restrict__ c_wtt, double* __restrict__ delta) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncoord) return;
    int lo = 0, hi = b;   // largest ci with cptr[ci] <= t
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (cptr[mid] <= t) lo = mid; else hi = mid;
    }
    const int ci = lo;
    const int64_t p = c_p[t];
    const double wcc = WJJ[(int64_t)ci * jp + ci];
    const double wtc = WJJ[p * jp + ci];
    const double wtt = WJJ[p * jp + p];
    const double a = (p == ci) ? wcc * wcc : wtc * wtc + wtt * wcc;
    c_ci[t] = ci;
    c_a[t] = a;
    c_inva[t] = 1.0 / a;
    c_wtc[t] = wtc;
    c_wtt[t] = wtt;
    delta[t] = 0.0;
}

template <bool U_IN_LDS>
__global__ __launch_bounds__(CD_THREADS) void k_cd(
    int jp, int b, const int64_t* __restrict__ cptr, const int32_t* __restrict__ c_p,
    const double* __restrict__ c_S, const double* __restrict__ c_A,
    const double* __restrict__ c_inva, const double* __restrict__ c_wtc,
    const double* __restrict__ WJJ, double lam, int max_sweeps, double tol,
    double* __restrict__ U, double* __restrict__ delta, double* __restrict__ mu_col,
    double* __restrict__ ug, double* __restrict__ stats) {
    extern __shared__ double sm[];
    double* zs = sm;                          // [CD_CHUNK]
    double* wcs = zs + CD_CHUNK;              // [CD_CHUNK]
    double* ws = wcs + CD_CHUNK;              // [CD_CHUNK][CD_WPAD]
    double* u = U_IN_LDS ? ws + CD_CHUNK * CD_WPAD : ug;   // [jp]
    __shared__ double s_red[CD_WAVES];
    __shared__ int s_stop;
    __shared__ double s_maxmu;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    int sweeps = 0;
    double maxmu = 0.0;
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        maxmu = 0.0;   // meaningful in wave 0
        for (int ci = 0; ci < b; ++ci) {
            const int64_t t0 = cptr[ci], t1 = cptr[ci + 1];
            if (t0 == t1) continue;
            for (int p = tid; p < jp; p += CD_THREADS) u[p] = U[(int64_t)p * b + ci];
            __syncthreads();
            const double wcc = WJJ[(int64_t)ci * jp + ci];
            for (int64_t k0 = t0; k0 < t1; k0 += CD_CHUNK) {
                const int K = (int)((t1 - k0) < CD_CHUNK ? (t1 - k0) : CD_CHUNK);
                // (2) dots z_k = W_{r_k, J'} . u
                for (int kk = wave; kk < K; kk += CD_WAVES) {
                    const double* row = WJJ + (int64_t)c_p[k0 + kk] * jp;
                    double s = 0.0;
                    for (int q = lane; q < jp; q += 64) s += row[q] * u[q];
                    s = wave_sum(s);
                    if (lane == 0) zs[kk] = s;
                }
                // W among the chunk's rows, and W_{r_k, c}
                for (int idx = tid; idx < K * K; idx += CD_THREADS) {
                    const int kk = idx / K, tt = idx - kk * K;
                    ws[kk * CD_WPAD + tt] =
                        WJJ[(int64_t)c_p[k0 + kk] * jp + c_p[k0 + tt]];
                }
                for (int kk = tid; kk < K; kk += CD_THREADS) wcs[kk] = c_wtc[k0 + kk];
                __syncthreads();
                // (3) the serial chain, one coordinate per step
                if (wave == 0) {
                    double z = lane < K ? zs[lane] : 0.0;
                    const double wk = lane < K ? wcs[lane] : 0.0;
                    for (int tt = 0; tt < K; ++tt) {
                        const int64_t t = k0 + tt;
                        const int p = c_p[t];
                        const double zt = readlane_d(z, tt);
                        const double wtc = c_wtc[t];
                        const double inva = c_inva[t];
                        const double bb = c_S[t] - wtc + zt;
                        const double d_old = delta[t];
                        const double x = c_A[t] + d_old;
                        const double y = x - bb * inva;
                        const double thr = lam * inva;
                        const double sh = y > thr ? y - thr : (y < -thr ? y + thr : 0.0);
                        const double mu = sh - x;
                        if (p != ci)
                            z += mu * (ws[lane * CD_WPAD + tt] * wcc + wk * wtc);
                        else
                            z += mu * wk * wcc;
                        if (lane == 0) {
                            delta[t] = d_old + mu;
                            mu_col[t] = mu;
                            u[p] += mu * wcc;
                            if (p != ci) u[ci] += mu * wtc;
                        }
                        maxmu = fmax(maxmu, fabs(mu));
                    }
                }
                __syncthreads();
            }
            // (4) fold the column's steps into U:  U_r += mu W_c,  U_c += mu W_r
            for (int q = tid; q < b; q += CD_THREADS) {
                const double wcq = WJJ[(int64_t)ci * jp + q];
                double acc = 0.0;
                for (int64_t t = t0; t < t1; ++t) {
                    const double mu = mu_col[t];
                    if (mu == 0.0) continue;
                    const int p = c_p[t];
                    if (p != ci) {
                        U[(int64_t)p * b + q] += mu * wcq;
                        acc += mu * WJJ[(int64_t)p * jp + q];
                    } else {
                        acc += mu * wcq;
                    }
                }
                U[(int64_t)ci * b + q] += acc;
            }
            __syncthreads();
        }
        // stopping rule: max|mu| <= tol * max|Delta|
        if (tid == 0) s_maxmu = maxmu;
        double dmax = 0.0;
        const int64_t nc = cptr[b];
        for (int64_t t = tid; t < nc; t += CD_THREADS) dmax = fmax(dmax, fabs(delta[t]));
        dmax = wave_max(dmax);
        if (lane == 0) s_red[wave] = dmax;
        __syncthreads();
        if (tid == 0) {
            double m = 0.0;
            for (int w = 0; w < CD_WAVES; ++w) m = fmax(m, s_red[w]);
            s_stop = (s_maxmu <= tol * m) ? 1 : 0;
            stats[1] = s_maxmu;
            stats[2] = m;
        }
        __syncthreads();
        ++sweeps;
        if (s_stop) break;
    }
    if (tid == 0) stats[0] = (double)sweeps;
}

}  // namespace

size_t cd_lds_bytes(int jp, bool u_in_lds) {
    return sizeof(double) * ((size_t)2 * CD_CHUNK + (size_t)CD_CHUNK * CD_WPAD +
                             (u_in_lds ? (size_t)jp : 0));
}

void launch_cd_prep(const int64_t* cptr, int b, int64_t ncoord, const int32_t* c_p,
                    const double* WJJ, int jp, int32_t* c_ci, double* c_a, double* c_inva,
                    double* c_wtc, double* c_wtt, double* delta, hipStream_t s) {
    if (ncoord <= 0) return;
    hipLaunchKernelGGL(k_cd_prep, dim3((unsigned)((ncoord + 255) / 256)), dim3(256), 0, s, cptr, b,
                       ncoord, c_p, WJJ, jp, c_ci, c_a, c_inva, c_wtc, c_wtt, delta);
    SIC_CHECK_LAUNCH();
}

void launch_cd(int jp, int b, const int64_t* cptr, const int32_t* c_p, const double* c_S,
               const double* c_A, const double* c_inva, const double* c_wtc, const double* WJJ,
               double lam, int max_sweeps, double tol, double* U, double* delta, double* mu_col,
               double* ug, double* stats, hipStream_t s) {
    const size_t lds_full = cd_lds_bytes(jp, true);
    const bool in_lds = lds_full <= CD_MAX_LDS_BYTES;
    const size_t lds = cd_lds_bytes(jp, in_lds);
    if (in_lds) {
        static bool attr_set = false;
        if (!attr_set) {
            SIC_HIP(hipFuncSetAttribute((const void*)k_cd<true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)CD_MAX_LDS_BYTES));
            attr_set = true;
        }
        hipLaunchKernelGGL(k_cd<true>, dim3(1), dim3(CD_THREADS), lds, s, jp, b, cptr, c_p, c_S,
                           c_A, c_inva, c_wtc, WJJ, lam, max_sweeps, tol, U, delta, mu_col, ug,
                           stats);
    } else {
        hipLaunchKernelGGL(k_cd<false>, dim3(1), dim3(CD_THREADS), lds, s, jp, b, cptr, c_p, c_S,
                           c_A, c_inva, c_wtc, WJJ, lam, max_sweeps, tol, U, delta, mu_col, ug,
                           stats);
    }
    SIC_CHECK_LAUNCH();
}

}  // namespace sic
