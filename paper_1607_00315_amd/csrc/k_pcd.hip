// Newton direction of one block by parallel coordinate descent accelerated by
// non-linear conjugate gradients (PCD-CG, Section 6.1.1), for blocks whose
// free set is too large for the sequential coordinate chain.
//
// The block model (Section 5.1 eq. (Quad_MLE_l1_prior) restricted by eq.
// (sub_Quad_MLE_l1_prior)) over the free coordinates k = (r_k, c_k) is
//   q(Delta) = sum_k gam_k [ g_k Delta_k + lam |A_k + Delta_k| ] + 0.5 tr(W Delta W Delta)
// with gam_k = 2 off the diagonal (Delta_rc = Delta_cr), 1 on it, and
// g_k = S_k - W_k. Its gradient at coordinate k is gam_k (g_k + z_k) with
// z = W Delta W on the free set, and its diagonal curvature gam_k a_k with a_k
// the 1-D coefficient of the coordinate-descent rule.
//
// One iteration:
//   1. PCD direction (Section 2, eq. (IST_direction) with D = diag of the
//      Hessian): every coordinate takes the 1-D minimiser of its own model at
//      the current z, d_k = median(-(b_k + lam)/a_k, -x_k, -(b_k - lam)/a_k),
//      with b_k = g_k + z_k and x_k = A_k + Delta_k;
//   2. conjugate direction p = d + beta p_prev, beta = max(0, <d, d - d_prev> /
//      <d_prev, d_prev>) in the gam-weighted inner product (Polak-Ribiere with
//      restarts), beta = 0 after a failed line search;
//   3. the Hessian product zp = W P W on the free set (P the symmetric matrix of
//      p), computed as Y = W_{J'J'} P_{J',I} (a sparse combination of rows of
//      W), then zp_k = Y[r_k].W[c_k] + W[r_k].(Y[c_k] - pdiag * W[c_k]) over
//      the block columns (pdiag: p on each column's diagonal coordinate);
//   4. line search on the exact model along p: the best of 64 step sizes on a
//      geometric grid (ratio 2^(1/8)) centred on the last accepted step; the
//      model change is sum_k gam_k [alpha p_k b_k + lam (|x_k + alpha p_k| - |x_k|)]
//      + alpha^2 C / 2 with C = <p, zp>, the first sum taken term by term per
//      candidate (near the minimiser b_k is close to -lam sign(x_k) and the
//      steps are far below |x_k|: separate sums would cancel); no candidate
//      below q(Delta) means alpha = 0 and a restart;
//   5. Delta += alpha p, z += alpha zp (z stays exact: the model is quadratic).
// The iteration stops when max |alpha p| <= tol * max |Delta| (the inner
// precision of Section 8, measured as the coordinate-descent sweeps measure
// it), or when a restart makes no progress, or at max_iter.
//
// Every step is a grid-wide kernel; the scalars live in device memory and the
// host only reads the stop flag every few iterations. No atomics: the result
// does not depend on scheduling.
#include "profiler.h"

namespace sic {

namespace {

constexpr int PT = 256;           // threads per workgroup
constexpr int PGRID = 1024;       // largest grid of the coordinate-parallel kernels
constexpr int NCAND = 64;         // line-search candidates (one per lane)
constexpr int YCOLS = 16;         // block columns per workgroup of the Y kernel
constexpr int DIRP = 5;           // partials per workgroup of the direction kernel
constexpr int ZPP = 3 + NCAND;    // partials per workgroup of the product kernel

enum { SC_ALPHA, SC_CENTER, SC_BETA, SC_DONE, SC_RESTART, SC_ITERS, SC_STEP, SC_DMAX, SC_COUNT };

__device__ inline double wsum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// |x + s| - |x|, exact when x + s keeps the sign of x (it is then +-s): near
// the minimiser the steps are many orders below |x|, and differencing two sums
// of |x| would lose them to rounding.
__device__ inline double l1_change(double x, double s) {
    const double y = x + s;
    if (x > 0.0 && y >= 0.0) return s;
    if (x < 0.0 && y <= 0.0) return -s;
    return fabs(y) - fabs(x);
}

__device__ inline double wmax(double v) {
    for (int off = 32; off > 0; off >>= 1) v = fmax(v, __shfl_xor(v, off, 64));
    return v;
}

// Step 5 for the previous iteration, then step 1 and the partial inner
// products of step 2 and of the stop test. final_pass: step 5 for the last
// accepted step (when the iteration cap ended the loop), then every coordinate
// whose own 1-D minimiser is zero (x + d = 0) is set to exactly zero: the
// conjugate combination and the grid step leave zeros inexact.
__global__ __launch_bounds__(PT) void k_pcd_dir(
    int64_t nc, const int32_t* __restrict__ c_p, const int32_t* __restrict__ c_ci,
    const double* __restrict__ c_S, const double* __restrict__ c_A,
    const double* __restrict__ c_wtc, const double* __restrict__ c_inva, double lam,
    double* __restrict__ delta, double* __restrict__ z, const double* __restrict__ p_old,
    const double* __restrict__ zp_old, const double* __restrict__ d_old,
    double* __restrict__ d_new, const double* __restrict__ sc, double* __restrict__ part,
    int final_pass) {
    const bool done = sc[SC_DONE] != 0.0;
    if (done && !final_pass) return;
    const double alpha = done ? 0.0 : sc[SC_ALPHA];
    double s_dd = 0.0, s_dD = 0.0, s_DD = 0.0, m_step = 0.0, m_D = 0.0;
    const int64_t stride = (int64_t)gridDim.x * PT;
    for (int64_t t = (int64_t)blockIdx.x * PT + threadIdx.x; t < nc; t += stride) {
        double D = delta[t], zz = z[t];
        if (alpha != 0.0) {
            const double pt = p_old[t];
            D += alpha * pt;
            zz += alpha * zp_old[t];
            delta[t] = D;
            z[t] = zz;
            m_step = fmax(m_step, fabs(alpha * pt));
        }
        m_D = fmax(m_D, fabs(D));
        const double x = c_A[t] + D;
        const double bb = c_S[t] - c_wtc[t] + zz;
        const double ia = c_inva[t];
        const double lo = -(bb + lam) * ia, hi = -(bb - lam) * ia;
        if (final_pass) {
            if (lo <= -x && -x <= hi) delta[t] = -c_A[t];
            continue;
        }
        const double d = fmax(lo, fmin(hi, -x));
        d_new[t] = d;
        const double g = c_p[t] == c_ci[t] ? 1.0 : 2.0;
        const double dp = d_old[t];
        s_dd += g * d * d;
        s_dD += g * d * dp;
        s_DD += g * dp * dp;
    }
    __shared__ double red[PT / 64][DIRP];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    s_dd = wsum(s_dd);
    s_dD = wsum(s_dD);
    s_DD = wsum(s_DD);
    m_step = wmax(m_step);
    m_D = wmax(m_D);
    if (lane == 0) {
        red[w][0] = s_dd;
        red[w][1] = s_dD;
        red[w][2] = s_DD;
        red[w][3] = m_step;
        red[w][4] = m_D;
    }
    __syncthreads();
    if (threadIdx.x < DIRP) {
        const int q = threadIdx.x;
        double v = red[0][q];
        for (int k = 1; k < PT / 64; ++k) v = q < 3 ? v + red[k][q] : fmax(v, red[k][q]);
        part[(int64_t)blockIdx.x * DIRP + q] = v;
    }
}

// Step 2's beta and the stop test (one workgroup).
__global__ __launch_bounds__(64) void k_pcd_beta(int nwg, const double* __restrict__ part,
                                                 double tol, double* __restrict__ sc) {
    if (sc[SC_DONE] != 0.0) return;
    const int q = threadIdx.x;
    __shared__ double v[DIRP];
    if (q < DIRP) {
        double a = part[q];
        for (int k = 1; k < nwg; ++k)
            a = q < 3 ? a + part[(int64_t)k * DIRP + q] : fmax(a, part[(int64_t)k * DIRP + q]);
        v[q] = a;
    }
    __syncthreads();
    if (q != 0) return;
    const double iters = sc[SC_ITERS];
    const double alpha_old = sc[SC_ALPHA];
    double done = 0.0;
    if (iters > 0.0) {
        if (alpha_old != 0.0 && v[3] <= tol * v[4]) done = 1.0;
        if (alpha_old == 0.0 && sc[SC_BETA] == 0.0) done = 1.0;   // a restart made no progress
    }
    sc[SC_STEP] = v[3];
    sc[SC_DMAX] = v[4];
    if (done != 0.0) {
        sc[SC_DONE] = 1.0;
        return;
    }
    double beta = 0.0;
    if (sc[SC_RESTART] == 0.0 && v[2] > 0.0) beta = fmax(0.0, (v[0] - v[1]) / v[2]);
    sc[SC_BETA] = beta;
    sc[SC_RESTART] = 0.0;
    sc[SC_ITERS] = iters + 1.0;
}

// Step 2's p = d + beta p_old and the first half of step 3: Y = W_{J'J'} P_{J',I}
// (jp x b, row-major), Y[r][s] = sum_{t in column s} p_t W[r_t][r]. Workgroup
// (column tile, row chunk); the row chunk 0 workgroups also store p and pdiag.
__global__ __launch_bounds__(PT) void k_pcd_y(
    int jp, int b, const int64_t* __restrict__ cptr, const int32_t* __restrict__ c_p,
    const int32_t* __restrict__ dg, const double* __restrict__ WJJ,
    const double* __restrict__ d_new, const double* __restrict__ p_old,
    double* __restrict__ p_new, double* __restrict__ pdiag, double* __restrict__ Y,
    const double* __restrict__ sc) {
    if (sc[SC_DONE] != 0.0) return;
    const double beta = sc[SC_BETA];
    const int s0 = blockIdx.x * YCOLS;
    const int ncol = min(YCOLS, b - s0);
    const int r = blockIdx.y * PT + threadIdx.x;
    const int rr = r < jp ? r : jp - 1;   // clamped: loads stay in bounds, stores are masked
    double acc[YCOLS];
#pragma unroll
    for (int j = 0; j < YCOLS; ++j) acc[j] = 0.0;
#pragma unroll
    for (int j = 0; j < YCOLS; ++j) {
        if (j < ncol) {
            const int64_t t1 = cptr[s0 + j + 1];
            int64_t t = cptr[s0 + j];
            for (; t + 8 <= t1; t += 8) {
                double wv[8], pv[8];
#pragma unroll
                for (int u = 0; u < 8; ++u) {
                    pv[u] = d_new[t + u] + beta * p_old[t + u];
                    wv[u] = WJJ[(int64_t)c_p[t + u] * jp + rr];
                }
#pragma unroll
                for (int u = 0; u < 8; ++u) acc[j] += pv[u] * wv[u];
            }
            for (; t < t1; ++t) acc[j] += (d_new[t] + beta * p_old[t]) * WJJ[(int64_t)c_p[t] * jp + rr];
        }
    }
    if (r < jp) {
        double* yr = Y + (int64_t)r * b + s0;
#pragma unroll
        for (int j = 0; j < YCOLS; ++j)
            if (j < ncol) yr[j] = acc[j];
    }
    if (blockIdx.y == 0) {
        const int64_t t0 = cptr[s0], t1 = cptr[s0 + ncol];
        for (int64_t t = t0 + threadIdx.x; t < t1; t += PT) p_new[t] = d_new[t] + beta * p_old[t];
        if (threadIdx.x < ncol) {
            const int s = s0 + threadIdx.x;
            const int k = dg[s];
            pdiag[s] = k >= 0 ? d_new[k] + beta * p_old[k] : 0.0;
        }
    }
}

// Second half of step 3 (zp on every coordinate, one wave per coordinate) and
// the partial sums of step 4: B, C and the change of the l1 sum at every
// candidate (lane j holds candidate j).
__global__ __launch_bounds__(PT) void k_pcd_zp(
    int64_t nc, int jp, int b, const int32_t* __restrict__ c_p, const int32_t* __restrict__ c_ci,
    const double* __restrict__ c_S, const double* __restrict__ c_A,
    const double* __restrict__ c_wtc, const double* __restrict__ WJJ,
    const double* __restrict__ Y, const double* __restrict__ pdiag,
    const double* __restrict__ p_new, const double* __restrict__ delta,
    const double* __restrict__ z, double* __restrict__ zp_new, const double* __restrict__ sc,
    double lam, double* __restrict__ part) {
    if (sc[SC_DONE] != 0.0) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double alpha_j = sc[SC_CENTER] * exp2((double)(lane - NCAND / 2) * 0.125);
    const int64_t nwaves = (int64_t)gridDim.x * (PT / 64);
    double B = 0.0, C = 0.0, Lj = 0.0;
    for (int64_t k = (int64_t)blockIdx.x * (PT / 64) + w; k < nc; k += nwaves) {
        const int r = c_p[k], c = c_ci[k];
        const double* yr = Y + (int64_t)r * b;
        const double* yc = Y + (int64_t)c * b;
        const double* wr = WJJ + (int64_t)r * jp;
        const double* wc = WJJ + (int64_t)c * jp;
        double s = 0.0;
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int j = lane + 64 * u;
            const bool in = j < b;
            const int jj = in ? j : 0;
            const double a1 = yr[jj], a2 = wc[jj], a3 = wr[jj], a4 = yc[jj], a5 = pdiag[jj];
            if (in) s += a1 * a2 + a3 * (a4 - a5 * a2);
        }
        const double zp = wsum(s);
        if (lane == 0) zp_new[k] = zp;
        const double pk = p_new[k];
        const double x = c_A[k] + delta[k];
        const double bb = c_S[k] - c_wtc[k] + z[k];
        const double g = r == c ? 1.0 : 2.0;
        B += g * bb * pk;
        C += g * pk * zp;
        // the linear and l1 parts per coordinate: near the minimiser b is close
        // to -lam sign(x) and their sums would cancel
        const double sj = alpha_j * pk;
        Lj += g * (sj * bb + lam * l1_change(x, sj));
    }
    __shared__ double lj[PT / 64][NCAND];
    __shared__ double bc[PT / 64][3];
    lj[w][lane] = Lj;
    if (lane == 0) {
        bc[w][0] = B;
        bc[w][1] = C;
        bc[w][2] = 0.0;
    }
    __syncthreads();
    double* out = part + (int64_t)blockIdx.x * ZPP;
    if (threadIdx.x < NCAND) {
        double v = lj[0][threadIdx.x];
        for (int k = 1; k < PT / 64; ++k) v += lj[k][threadIdx.x];
        out[3 + threadIdx.x] = v;
    } else if (threadIdx.x < NCAND + 3) {
        const int q = threadIdx.x - NCAND;
        double v = bc[0][q];
        for (int k = 1; k < PT / 64; ++k) v += bc[k][q];
        out[q] = v;
    }
}

// Step 4's choice (one wave, one lane per candidate).
__global__ __launch_bounds__(64) void k_pcd_alpha(int nwg, const double* __restrict__ part,
                                                  double lam, double* __restrict__ sc) {
    if (sc[SC_DONE] != 0.0) return;
    const int j = threadIdx.x;
    double C = 0.0, Lj = 0.0;
    for (int k = 0; k < nwg; ++k) {
        const double* p = part + (int64_t)k * ZPP;
        C += p[1];
        Lj += p[3 + j];
    }
    const double a = sc[SC_CENTER] * exp2((double)(j - NCAND / 2) * 0.125);
    const double phi = Lj + 0.5 * a * a * C;   // q(Delta + a p) - q(Delta)
    // argmin over lanes, the smallest index on ties
    double best = phi;
    int bj = j;
    for (int off = 32; off > 0; off >>= 1) {
        const double ob = __shfl_xor(best, off, 64);
        const int oj = __shfl_xor(bj, off, 64);
        if (ob < best || (ob == best && oj < bj)) {
            best = ob;
            bj = oj;
        }
    }
    if (j == 0) {
        if (best < 0.0) {
            const double ab = sc[SC_CENTER] * exp2((double)(bj - NCAND / 2) * 0.125);
            sc[SC_ALPHA] = ab;
            sc[SC_CENTER] = ab;
        } else {
            sc[SC_ALPHA] = 0.0;
            sc[SC_RESTART] = 1.0;
        }
    }
}

__global__ void k_pcd_init(int64_t nc, int b, const int32_t* __restrict__ c_p,
                           const int32_t* __restrict__ c_ci, int32_t* __restrict__ dg,
                           double* __restrict__ z, double* __restrict__ p0,
                           double* __restrict__ zp0, double* __restrict__ d0,
                           double* __restrict__ sc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < b) dg[t] = -1;
    if (t < SC_COUNT) {
        double v = 0.0;
        if (t == SC_CENTER || t == SC_BETA || t == SC_RESTART) v = 1.0;
        sc[t] = v;
    }
    if (t < nc) {
        z[t] = 0.0;
        p0[t] = 0.0;
        zp0[t] = 0.0;
        d0[t] = 0.0;
    }
}

__global__ void k_pcd_diag(int64_t nc, const int32_t* __restrict__ c_p,
                           const int32_t* __restrict__ c_ci, int32_t* __restrict__ dg) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t < nc && c_p[t] == c_ci[t]) dg[c_ci[t]] = (int32_t)t;   // one diagonal per column
}

__global__ void k_pcd_stats(const double* __restrict__ sc, double* __restrict__ stats) {
    if (threadIdx.x == 0) {
        stats[0] = sc[SC_ITERS];
        stats[1] = sc[SC_STEP];
        for (int k = 2; k < 8; ++k) stats[k] = 0.0;
    }
}

}  // namespace

int64_t launch_pcd(int64_t nc, int jp, int b, const int64_t* cptr, const int32_t* c_p,
                   const int32_t* c_ci, const double* c_S, const double* c_A,
                   const double* c_wtc, const double* c_inva, const double* WJJ, double lam,
                   int max_iter, double tol, double* delta, PcdWork& wk, double* stats,
                   double* h_flag, hipStream_t s) {
    if (nc <= 0 || b < 1 || b > 256 || jp < b) throw SicError(SIC_EINTERNAL, "bad PCD-CG shape");
    const int grid = (int)std::min<int64_t>(PGRID, (nc + PT - 1) / PT);
    const int zgrid = (int)std::min<int64_t>(PGRID, (nc + PT / 64 - 1) / (PT / 64));
    wk.z.reserve(nc);
    wk.d[0].reserve(nc); wk.d[1].reserve(nc);
    wk.p[0].reserve(nc); wk.p[1].reserve(nc);
    wk.zp[0].reserve(nc); wk.zp[1].reserve(nc);
    wk.Y.reserve((size_t)jp * b);
    wk.pdiag.reserve(b);
    wk.dg.reserve(b);
    wk.part.reserve((size_t)std::max(grid * DIRP, zgrid * ZPP));
    wk.sc.reserve(SC_COUNT);
    const unsigned ig = (unsigned)((std::max<int64_t>(std::max<int64_t>(nc, b), SC_COUNT) + 255) / 256);
    hipLaunchKernelGGL(k_pcd_init, dim3(ig), dim3(256), 0, s, nc, b, c_p, c_ci, wk.dg.p, wk.z.p,
                       wk.p[0].p, wk.zp[0].p, wk.d[0].p, wk.sc.p);
    SIC_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_pcd_diag, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, nc, c_p,
                       c_ci, wk.dg.p);
    SIC_CHECK_LAUNCH();
    prof_begin(KK_PCD, s);
    int cur = 0;   // p[cur], zp[cur], d[cur] hold the previous iteration
    const dim3 ygrid((unsigned)((b + YCOLS - 1) / YCOLS), (unsigned)((jp + PT - 1) / PT));
    int it = 0;
    for (; it < max_iter; ++it) {
        const int nx = 1 - cur;
        hipLaunchKernelGGL(k_pcd_dir, dim3(grid), dim3(PT), 0, s, nc, c_p, c_ci, c_S, c_A, c_wtc,
                           c_inva, lam, delta, wk.z.p, wk.p[cur].p, wk.zp[cur].p, wk.d[cur].p,
                           wk.d[nx].p, wk.sc.p, wk.part.p, 0);
        hipLaunchKernelGGL(k_pcd_beta, dim3(1), dim3(64), 0, s, grid, wk.part.p, tol, wk.sc.p);
        hipLaunchKernelGGL(k_pcd_y, ygrid, dim3(PT), 0, s, jp, b, cptr, c_p, wk.dg.p, WJJ,
                           wk.d[nx].p, wk.p[cur].p, wk.p[nx].p, wk.pdiag.p, wk.Y.p, wk.sc.p);
        hipLaunchKernelGGL(k_pcd_zp, dim3(zgrid), dim3(PT), 0, s, nc, jp, b, c_p, c_ci, c_S, c_A,
                           c_wtc, WJJ, wk.Y.p, wk.pdiag.p, wk.p[nx].p, delta, wk.z.p,
                           wk.zp[nx].p, wk.sc.p, lam, wk.part.p);
        hipLaunchKernelGGL(k_pcd_alpha, dim3(1), dim3(64), 0, s, zgrid, wk.part.p, lam, wk.sc.p);
        SIC_CHECK_LAUNCH();
        cur = nx;
        if ((it & 3) == 3) {
            SIC_HIP(hipMemcpyAsync(h_flag, wk.sc.p + SC_DONE, sizeof(double), hipMemcpyDeviceToHost, s));
            stream_wait(s);
            if (*h_flag != 0.0) break;
        }
    }
    // the last accepted step when the iteration cap ended the loop, and exact zeros
    hipLaunchKernelGGL(k_pcd_dir, dim3(grid), dim3(PT), 0, s, nc, c_p, c_ci, c_S, c_A, c_wtc,
                       c_inva, lam, delta, wk.z.p, wk.p[cur].p, wk.zp[cur].p, wk.d[cur].p,
                       wk.d[1 - cur].p, wk.sc.p, wk.part.p, 1);
    hipLaunchKernelGGL(k_pcd_stats, dim3(1), dim3(64), 0, s, wk.sc.p, stats);
    SIC_CHECK_LAUNCH();
    // per iteration: the rows of W read for Y (8 jp bytes per coordinate), Y and
    // three b-rows per coordinate for zp, and the coordinate arrays
    const double bytes = 8.0 * (double)nc * jp + 8.0 * (double)nc * 4.0 * b + 8.0 * 12.0 * nc;
    return prof_end(KK_PCD, s, bytes, 2.0 * (double)nc * (jp + 3.0 * b));
}

}  // namespace sic
