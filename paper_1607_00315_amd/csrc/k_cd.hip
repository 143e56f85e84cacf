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
#include "profiler.h"

#include <mutex>

namespace sic {

namespace {

constexpr int CD_THREADS = 1024;
constexpr int CD_WAVES = CD_THREADS / 64;
constexpr int CD_CHUNK = 64;
constexpr int CD_WPAD = CD_CHUNK + 1;
constexpr int CD_COLCAP = 1024;   // steps of one column staged in LDS for the fold
constexpr int CD_MAXB = 256;      // largest block

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
    double* __restrict__ ug, unsigned char* __restrict__ markg, double* __restrict__ stats) {
    extern __shared__ double sm[];
    double* zs = sm;                              // [CD_CHUNK] dots of the chunk
    double* wcs = zs + CD_CHUNK;                  // [CD_CHUNK] W_{r_k, c}
    double* ws = wcs + CD_CHUNK;                  // [CD_CHUNK][CD_WPAD] W among the chunk
    double* cs_inva = ws + CD_CHUNK * CD_WPAD;    // [CD_CHUNK] chunk coordinate data
    double* cs_S = cs_inva + CD_CHUNK;
    double* cs_A = cs_S + CD_CHUNK;
    double* cs_d = cs_A + CD_CHUNK;
    int* cs_p = (int*)(cs_d + CD_CHUNK);          // [CD_CHUNK]
    double* colmu = cs_d + CD_CHUNK + CD_CHUNK / 2;   // [CD_COLCAP] steps of the column
    int* colp = (int*)(colmu + CD_COLCAP);        // [CD_COLCAP]
    double* wc_row = colmu + CD_COLCAP + CD_COLCAP / 2;   // [CD_MAXB] W_{c, I}
    double* u = U_IN_LDS ? wc_row + CD_MAXB : ug;         // [jp] U[:, c]
    unsigned char* mark = U_IN_LDS ? (unsigned char*)(u + jp) : markg;   // [jp]
    __shared__ double s_red[CD_WAVES];
    __shared__ int s_stop;
    __shared__ double s_maxmu;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);

    for (int q = tid; q < jp; q += CD_THREADS) mark[q] = 0;
    __syncthreads();
    int sweeps = 0;
    double maxmu = 0.0;
    // phase clocks (thread 0): u load, staging + dots, chain, fold
    long long tph[4] = {0, 0, 0, 0};
    long long tlast = wall_clock64();
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        maxmu = 0.0;   // meaningful in wave 0
        for (int ci = 0; ci < b; ++ci) {
            const int64_t t0 = cptr[ci], t1 = cptr[ci + 1];
            if (t0 == t1) continue;
            const int64_t kc = t1 - t0;
            // (1) u = U[:, c] and W_{c, I} into LDS
            for (int p = tid; p < jp; p += CD_THREADS) u[p] = U[(int64_t)p * b + ci];
            for (int q = tid; q < b; q += CD_THREADS) wc_row[q] = WJJ[(int64_t)ci * jp + q];
            __syncthreads();
            if (tid == 0) { const long long now = wall_clock64(); tph[0] += now - tlast; tlast = now; }
            const double wcc = wc_row[ci];
            for (int64_t k0 = t0; k0 < t1; k0 += CD_CHUNK) {
                const int K = (int)((t1 - k0) < CD_CHUNK ? (t1 - k0) : CD_CHUNK);
                // stage the chunk's coordinate data; mark its rows for the capture below
                if (tid < K) {
                    const int p = c_p[k0 + tid];
                    cs_p[tid] = p;
                    wcs[tid] = c_wtc[k0 + tid];
                    cs_inva[tid] = c_inva[k0 + tid];
                    cs_S[tid] = c_S[k0 + tid];
                    cs_A[tid] = c_A[k0 + tid];
                    cs_d[tid] = delta[k0 + tid];
                    mark[p] = (unsigned char)(tid + 1);
                }
                __syncthreads();
                // (2) dots z_k = W_{r_k, J'} u, eight independent loads in flight per
                //     lane; W among the chunk's rows is captured from the same rows
                for (int kk = wave; kk < K; kk += CD_WAVES) {
                    const double* row = WJJ + (int64_t)cs_p[kk] * jp;
                    double* wsk = ws + kk * CD_WPAD;
                    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
                    double a4 = 0.0, a5 = 0.0, a6 = 0.0, a7 = 0.0;
                    int q = lane;
                    for (; q + 7 * 64 < jp; q += 8 * 64) {
                        double r[8];
#pragma unroll
                        for (int i = 0; i < 8; ++i) r[i] = row[q + 64 * i];
                        a0 += r[0] * u[q];
                        a1 += r[1] * u[q + 64];
                        a2 += r[2] * u[q + 128];
                        a3 += r[3] * u[q + 192];
                        a4 += r[4] * u[q + 256];
                        a5 += r[5] * u[q + 320];
                        a6 += r[6] * u[q + 384];
                        a7 += r[7] * u[q + 448];
#pragma unroll
                        for (int i = 0; i < 8; ++i) {
                            const int mk = mark[q + 64 * i];
                            if (mk) wsk[mk - 1] = r[i];
                        }
                    }
                    for (; q < jp; q += 64) {
                        const double r = row[q];
                        a0 += r * u[q];
                        const int mk = mark[q];
                        if (mk) wsk[mk - 1] = r;
                    }
                    const double sdot = wave_sum(((a0 + a1) + (a2 + a3)) + ((a4 + a5) + (a6 + a7)));
                    if (lane == 0) zs[kk] = sdot;
                }
                __syncthreads();
                if (tid == 0) { const long long now = wall_clock64(); tph[1] += now - tlast; tlast = now; }
                // (3) the serial chain, one coordinate per step; coordinate k's data
                //     sits in lane k and is broadcast with readlane
                if (wave == 0) {
                    const bool on = lane < K;
                    double z = on ? zs[lane] : 0.0;
                    const double wk = on ? wcs[lane] : 0.0;
                    const int rp = on ? cs_p[lane] : 0;
                    const double rinva = on ? cs_inva[lane] : 0.0;
                    const double rS = on ? cs_S[lane] : 0.0;
                    const double rA = on ? cs_A[lane] : 0.0;
                    double rd = on ? cs_d[lane] : 0.0;
                    double rmu = 0.0;
                    double wnext = on ? ws[lane * CD_WPAD] : 0.0;
                    for (int tt = 0; tt < K; ++tt) {
                        const double wrow = wnext;
                        if (tt + 1 < K) wnext = on ? ws[lane * CD_WPAD + tt + 1] : 0.0;
                        const int p = __builtin_amdgcn_readlane(rp, tt);
                        const double zt = readlane_d(z, tt);
                        const double wtc = readlane_d(wk, tt);
                        const double inva = readlane_d(rinva, tt);
                        const double d_old = readlane_d(rd, tt);
                        const double x = readlane_d(rA, tt) + d_old;
                        const double bb = readlane_d(rS, tt) - wtc + zt;
                        const double y = x - bb * inva;
                        const double thr = lam * inva;
                        const double sh = y > thr ? y - thr : (y < -thr ? y + thr : 0.0);
                        const double mu = sh - x;
                        if (p != ci)
                            z += mu * (wrow * wcc + wk * wtc);
                        else
                            z += mu * wk * wcc;
                        if (lane == tt) {
                            rd = d_old + mu;
                            rmu = mu;
                        }
                        maxmu = fmax(maxmu, fabs(mu));
                    }
                    if (on) {
                        delta[k0 + lane] = rd;
                        mu_col[k0 + lane] = rmu;
                        const int64_t slot = k0 - t0 + lane;
                        if (slot < CD_COLCAP) {
                            colmu[slot] = rmu;
                            colp[slot] = rp;
                        }
                        // u_r += mu W_cc for every step (r = c on the diagonal step)
                        if (rmu != 0.0) u[rp] += rmu * wcc;
                    }
                    // u_c += sum over off-diagonal steps of mu W_rc
                    const double contrib = wave_sum((on && rp != ci) ? rmu * wk : 0.0);
                    if (lane == 0) u[ci] += contrib;
                }
                if (tid < K) mark[cs_p[tid]] = 0;
                __syncthreads();
                if (tid == 0) { const long long now = wall_clock64(); tph[2] += now - tlast; tlast = now; }
            }
            // (4) fold the column's steps into U:  U_r += mu W_c for rows r != c, one
            //     independent update per (coordinate, block column) pair, and
            //     U_c += sum_t mu_t W_{r_t} with four partial sums per block column
            {
                const bool in_lds = kc <= CD_COLCAP;
#pragma unroll 4
                for (int64_t idx = tid; idx < kc * b; idx += CD_THREADS) {
                    const int64_t t = idx / b;
                    const int q = (int)(idx - t * b);
                    const double mu = in_lds ? colmu[t] : mu_col[t0 + t];
                    const int p = in_lds ? colp[t] : c_p[t0 + t];
                    if (mu != 0.0 && p != ci) U[(int64_t)p * b + q] += mu * wc_row[q];
                }
                const int h = tid / CD_MAXB, q = tid - h * CD_MAXB;
                double acc = 0.0;
                if (q < b) {
#pragma unroll 4
                    for (int64_t t = h; t < kc; t += CD_THREADS / CD_MAXB) {
                        const double mu = in_lds ? colmu[t] : mu_col[t0 + t];
                        const int p = in_lds ? colp[t] : c_p[t0 + t];
                        if (mu != 0.0) acc += mu * WJJ[(int64_t)p * jp + q];
                    }
                }
                ws[h * CD_MAXB + q] = acc;
                __syncthreads();
                if (h == 0 && q < b) {
                    double sacc = 0.0;
                    for (int g2 = 0; g2 < CD_THREADS / CD_MAXB; ++g2) sacc += ws[g2 * CD_MAXB + q];
                    U[(int64_t)ci * b + q] += sacc;
                }
            }
            __syncthreads();
            if (tid == 0) { const long long now = wall_clock64(); tph[3] += now - tlast; tlast = now; }
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
    if (tid == 0) {
        stats[0] = (double)sweeps;
        for (int i = 0; i < 4; ++i) stats[3 + i] = (double)tph[i];
    }
}


// ------------------------------------------------------------------------
// Explicit coordinate Hessian form of the same sweep.
//
// With Delta = 0 at the start, z_k = (W Delta W)_{r_k c_k} starts at zero and
// a step mu_t on coordinate t = (r_t, c_t) changes every z_k by mu_t H[k][t],
//   H[k][t] = W_{r_k r_t} W_{c_t c_k} + [r_t != c_t] W_{r_k c_t} W_{r_t c_k},
// the coefficient of Delta_t in the model gradient of coordinate k
// (H[t][t] = a_t). Building H once per block turns a sweep into
//   for each chunk of 64 consecutive coordinates (the same visiting order):
//     one wave runs the 64 steps, correcting the chunk's own z in registers
//     from the 64 x 64 diagonal tile of H held in LDS,
//   then every other z_k receives sum_t H[k][t] mu_t from one pass over the
//     chunk's 64 columns of H (coalesced rows of H^T, zero steps skipped).
// No U = Delta W is kept, so nothing is staged or folded per block column.

constexpr int CDH_THREADS = 1024;
constexpr int CDH_WAVES = CDH_THREADS / 64;
constexpr int CDH_K = 64;   // chunk length = wave size

// Barrier for LDS traffic only: outstanding global loads (prefetches into
// registers) stay in flight across it.
__device__ inline void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// HT[t * nc + k] = H[k][t] (column t of H stored contiguously), formed in
// float64 and stored as HV (float64, or float for the reduced-precision cycles).
template <typename HV>
__global__ void k_cd_hess(int64_t nc, int jp, const int32_t* __restrict__ c_p,
                          const int32_t* __restrict__ c_ci, const double* __restrict__ WJJ,
                          HV* __restrict__ HT) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t t = blockIdx.y;
    if (k >= nc) return;
    const int pt = c_p[t], ct = c_ci[t];
    const int pk = c_p[k], ck = c_ci[k];
    const double* wpt = WJJ + (int64_t)pt * jp;
    const double* wct = WJJ + (int64_t)ct * jp;
    double h = wpt[pk] * wct[ck];
    if (pt != ct) h += wct[pk] * wpt[ck];
    HT[t * nc + k] = (HV)h;
}

// p[idx] when cond, else dflt, with the load itself unconditional (index 0
// when !cond, which must be a valid element): a predicated load would become
// a branch that waits for its data before the next load is issued.
template <typename T>
__device__ inline double load_or(const T* __restrict__ p, int64_t idx, bool cond, double dflt) {
    const double v = (double)p[cond ? idx : 0];
    return cond ? v : dflt;
}

constexpr int CDH_RMAX = 4;    // coordinate rows per thread in the Hessian products (4096 / 1024)
constexpr int CDH_PAD = 16;    // the nonzero-step list is zero padded to a multiple of this

// One coordinate step of the chain, on lane data broadcast from lane tt:
// y = x - (S - W_rc + z)/a = p - z/a, soft(y) = y - clamp(y, -lam/a, lam/a),
// mu = soft(y) - x; every lane then adds mu H[k][tt] to its own z.
__device__ __forceinline__ void cd_step(int tt, double p, double ia, double thr, double xl, double h,
                                        int lane, double& z, double& mul, double& maxmu) {
    const double zt = readlane_d(z, tt);
    const double pt = readlane_d(p, tt), iat = readlane_d(ia, tt);
    const double tht = readlane_d(thr, tt), xt = readlane_d(xl, tt);
    const double y = pt - zt * iat;
    const double c = fmax(fmin(y, tht), -tht);
    const double mu = (y - c) - xt;
    z += mu * h;
    if (lane == tt) mul = mu;
    maxmu = fmax(maxmu, fabs(mu));
}

template <int ROWS>   // coordinate rows per thread: ceil(nc / 1024)
__global__ __launch_bounds__(CDH_THREADS) void k_cd_dense(
    int64_t nc, const double* __restrict__ HT, const double* __restrict__ c_S,
    const double* __restrict__ c_A, const double* __restrict__ c_inva,
    const double* __restrict__ c_wtc, double lam, int max_sweeps, double tol,
    double* __restrict__ delta, double* __restrict__ stats) {
    extern __shared__ double sm[];
    double* zs = sm;                    // [nc] z = (W Delta W) on the coordinates
    double* ds = zs + nc;               // [nc] Delta
    double* Hc = ds + nc;               // [CDH_K][CDH_K] diagonal tile of the chunk, [t][k]
    double* nzm = Hc + CDH_K * CDH_K;   // [CDH_K] nonzero steps of the chunk (zero padded)
    int* nzl = (int*)(nzm + CDH_K);     // [CDH_K] their chunk positions
    __shared__ double s_red[CDH_WAVES];
    __shared__ int s_nnz, s_stop;
    __shared__ double s_maxmu;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int nchunks = (int)((nc + CDH_K - 1) / CDH_K);

    for (int64_t k = tid; k < nc; k += CDH_THREADS) {
        zs[k] = 0.0;
        ds[k] = 0.0;
    }
    // register copy of the next chunk's diagonal tile (entry e = t * 64 + k)
    constexpr int HPT = CDH_K * CDH_K / CDH_THREADS;
    double hreg[HPT];
    auto load_tile = [&](int ch) {
        const int64_t k0 = (int64_t)ch * CDH_K;
        const int K = (int)((nc - k0) < CDH_K ? (nc - k0) : CDH_K);
#pragma unroll
        for (int j = 0; j < HPT; ++j) {
            const int e = tid + CDH_THREADS * j;
            const int t = e / CDH_K, k = e % CDH_K;
            hreg[j] = load_or(HT, (k0 + t) * nc + k0 + k, t < K && k < K, 0.0);
        }
    };
    // wave 0: the next chunk's per-coordinate constants, one coordinate per lane
    double nS = 0.0, nW = 0.0, nA = 0.0, ninva = 0.0;
    auto load_lane = [&](int ch) {
        const int64_t k = (int64_t)ch * CDH_K + lane;
        const bool on = k < nc;
        nS = load_or(c_S, k, on, 0.0);
        nW = load_or(c_wtc, k, on, 0.0);
        nA = load_or(c_A, k, on, 0.0);
        ninva = load_or(c_inva, k, on, 0.0);
    };
    load_tile(0);
    if (wave == 0) load_lane(0);

    int sweeps = 0;
    double maxmu = 0.0;   // meaningful in wave 0
    long long tph[3] = {0, 0, 0};   // thread 0: chain, Hessian products, staging waits
    long long tlast = wall_clock64();
    for (int sweep = 0; sweep < max_sweeps; ++sweep) {
        maxmu = 0.0;
        for (int ch = 0; ch < nchunks; ++ch) {
            const int64_t k0 = (int64_t)ch * CDH_K;
            const int K = (int)((nc - k0) < CDH_K ? (nc - k0) : CDH_K);
            const int nch = ch + 1 < nchunks ? ch + 1 : 0;
#pragma unroll
            for (int j = 0; j < HPT; ++j) Hc[tid + CDH_THREADS * j] = hreg[j];
            lds_barrier();   // tile, z and Delta of the chunk are in place
            if (tid == 0) { const long long now = wall_clock64(); tph[2] += now - tlast; tlast = now; }
            load_tile(nch);  // in flight during the chain and the products
            if (wave == 0) {
                // lanes >= K carry zeros: their steps are exactly 0 and change nothing
                const bool on = lane < K;
                const int kl = on ? (int)k0 + lane : (int)k0;
                const double ia = on ? ninva : 0.0;
                const double d0 = on ? ds[kl] : 0.0;
                const double xl = on ? nA + d0 : 0.0;
                const double p = on ? xl - (nS - nW) * ia : 0.0;
                const double thr = lam * ia;
                double z = on ? zs[kl] : 0.0;
                load_lane(nch);
                double mul = 0.0;
                const int K4 = (K + 3) & ~3;
                for (int tt = 0; tt < K4; tt += 4) {
                    const double h0 = Hc[tt * CDH_K + lane], h1 = Hc[(tt + 1) * CDH_K + lane];
                    const double h2 = Hc[(tt + 2) * CDH_K + lane], h3 = Hc[(tt + 3) * CDH_K + lane];
                    cd_step(tt, p, ia, thr, xl, h0, lane, z, mul, maxmu);
                    cd_step(tt + 1, p, ia, thr, xl, h1, lane, z, mul, maxmu);
                    cd_step(tt + 2, p, ia, thr, xl, h2, lane, z, mul, maxmu);
                    cd_step(tt + 3, p, ia, thr, xl, h3, lane, z, mul, maxmu);
                }
                if (on) {
                    zs[kl] = z;
                    ds[kl] = d0 + mul;
                }
                // compacted nonzero steps, zero padded to a multiple of the batch
                const bool nzs = on && mul != 0.0;
                const unsigned long long nzm_bits = __ballot(nzs);
                const int nnz = __popcll(nzm_bits);
                if (nzs) {
                    const int pos = __popcll(nzm_bits & ((1ull << lane) - 1ull));
                    nzl[pos] = lane;
                    nzm[pos] = mul;
                }
                const int npad = (nnz + CDH_PAD - 1) / CDH_PAD * CDH_PAD;
                if (lane >= nnz && lane < npad) {
                    nzl[lane] = 0;
                    nzm[lane] = 0.0;
                }
                if (lane == 0) s_nnz = nnz;
            }
            lds_barrier();   // steps of the chunk are in place
            if (tid == 0) { const long long now = wall_clock64(); tph[0] += now - tlast; tlast = now; }
            // z_k += sum_t H[k][t] mu_t for every coordinate outside the chunk; a
            // thread's rows k = tid + 1024 r load their batches together
            const int nnz = s_nnz;
            if (nnz > 0) {
                constexpr int BATCH = ROWS == 1 ? 16 : (ROWS == 2 ? 8 : 4);   // 16 loads in flight
                const int npad = (nnz + CDH_PAD - 1) / CDH_PAD * CDH_PAD;
                const double* hcol = HT + k0 * nc;
                double acc[ROWS];
                bool rv[ROWS];
                int64_t rk[ROWS];
#pragma unroll
                for (int r = 0; r < ROWS; ++r) {
                    const int64_t k = tid + (int64_t)CDH_THREADS * r;
                    rv[r] = k < nc && !(k >= k0 && k < k0 + K);
                    rk[r] = rv[r] ? k : 0;
                    acc[r] = 0.0;
                }
                for (int i = 0; i < npad; i += BATCH) {
                    double hv[ROWS][BATCH];
#pragma unroll
                    for (int r = 0; r < ROWS; ++r)
#pragma unroll
                        for (int q = 0; q < BATCH; ++q)
                            hv[r][q] = hcol[(int64_t)nzl[i + q] * nc + rk[r]];
#pragma unroll
                    for (int r = 0; r < ROWS; ++r)
#pragma unroll
                        for (int q = 0; q < BATCH; ++q) acc[r] += hv[r][q] * nzm[i + q];
                }
#pragma unroll
                for (int r = 0; r < ROWS; ++r)
                    if (rv[r]) zs[rk[r]] += acc[r];
            }
            if (tid == 0) { const long long now = wall_clock64(); tph[1] += now - tlast; tlast = now; }
        }
        // stopping rule: max|mu| <= tol * max|Delta|
        if (tid == 0) s_maxmu = maxmu;
        double dmax = 0.0;
        for (int64_t k = tid; k < nc; k += CDH_THREADS) dmax = fmax(dmax, fabs(ds[k]));
        dmax = wave_max(dmax);
        if (lane == 0) s_red[wave] = dmax;
        lds_barrier();
        if (tid == 0) {
            double m = 0.0;
            for (int w = 0; w < CDH_WAVES; ++w) m = fmax(m, s_red[w]);
            s_stop = (s_maxmu <= tol * m) ? 1 : 0;
            stats[1] = s_maxmu;
            stats[2] = m;
        }
        lds_barrier();
        ++sweeps;
        if (s_stop) break;
    }
    for (int64_t k = tid; k < nc; k += CDH_THREADS) delta[k] = ds[k];
    if (tid == 0) {
        stats[0] = (double)sweeps;
        for (int i = 0; i < 3; ++i) stats[3 + i] = (double)tph[i];
        stats[6] = 0.0;
    }
}


// ------------------------------------------------------------------------
// Pipelined explicit-Hessian sweep (blocks whose z, Delta and four 64 x 64
// tiles fit in LDS). Chunk intervals g = 0, 1, ... (chunk i = g mod C):
//   wave 0     applies the previous chunk's steps to the rows of chunk i from
//              the prefetched tile H[chunk i][chunk i-1], then runs the
//              chain of chunk i on the tile H[chunk i][chunk i] and publishes
//              its nonzero steps;
//   waves 1-15 apply the previous chunk's steps to every row outside chunks
//              i-1 and i (streaming those columns of H^T) and prefetch the
//              two tiles of the next interval.
// One barrier per chunk; tiles and step lists are double buffered. The rows
// of chunk i receive every step before its chain: steps of chunk i-1 from
// wave 0, older ones from the workers' earlier intervals.
constexpr int CDP_THREADS = 1024;
constexpr int CDP_WORKERS = CDP_THREADS - 64;
constexpr int CDP_TILE = CDH_K * CDH_K;
constexpr int CDP_CONST = 4 * CDH_K;   // a chunk's 1/a, A, S and W_rc, staged with its tiles
constexpr int CDP_TPT = (2 * CDP_TILE + CDP_CONST + CDP_WORKERS - 1) / CDP_WORKERS;   // prefetch loads per worker
// The step list is zero padded to a multiple of this, the column loads a worker
// has in flight at once
constexpr int CDP_PAD = 16;

__device__ __forceinline__ double cd_soft(double y, double t) {
    return y > t ? y - t : (y < -t ? y + t : 0.0);
}

template <int ROWS, typename HV>   // worker rows per thread: ceil(nc / 960); H's storage type
__global__ __launch_bounds__(CDP_THREADS) void k_cd_pipe(
    int64_t nc, const HV* __restrict__ HT, const double* __restrict__ c_S,
    const double* __restrict__ c_A, const double* __restrict__ c_inva,
    const double* __restrict__ c_wtc, double lam, int max_sweeps, double tol,
    double* __restrict__ delta, double* __restrict__ stats) {
    extern __shared__ double sm[];
    double* zs = sm;                          // [nc]
    double* ds = zs + nc;                     // [nc]
    double* Dt = ds + nc;                     // [2][64 x 64] H[chunk i][chunk i], [t][k]
    double* St = Dt + 2 * CDP_TILE;           // [2][64 x 64] H[chunk i][chunk i-1], [t][k]
    double* mud = St + 2 * CDP_TILE;          // [2][64] steps of the chunk, dense (0 when none)
    double* nzm = mud + 2 * CDH_K;            // [2][64] nonzero steps (zero padded)
    double* cst = nzm + 2 * CDH_K;            // [2][4][64] chunk i's 1/a, A, S, W_rc
    int* nzl = (int*)(cst + 2 * CDP_CONST);   // [2][64] their chunk positions
    __shared__ int s_nnz[2];
    __shared__ int s_stop;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int C = (int)((nc + CDH_K - 1) / CDH_K);
    auto klen = [&](int c) {
        const int64_t r = nc - (int64_t)c * CDH_K;
        return (int)(r < CDH_K ? r : CDH_K);
    };
    // worker: load the tiles of chunk ci (and its predecessor cp) and the
    // constants of chunk ci into registers
    double treg[CDP_TPT];
    auto load_tiles = [&](int ci, int cp) {
        const int64_t ki = (int64_t)ci * CDH_K, kp = (int64_t)cp * CDH_K;
        const int Ki = klen(ci), Kp = klen(cp);
#pragma unroll
        for (int r = 0; r < CDP_TPT; ++r) {
            // unconditional loads: a tile entry (element 0 of H past the tiles,
            // discarded), and in the slot that reaches past the tiles a constant
            const int e = (tid - 64) + CDP_WORKERS * r;
            const bool is_tile = e < 2 * CDP_TILE;
            const int which = e / CDP_TILE, f = e % CDP_TILE;
            const int t = f / CDH_K, k = f % CDH_K;
            const bool dtile = which == 0;
            const int64_t col = (dtile ? ki : kp) + t;
            const bool ok = is_tile && k < Ki && (dtile ? t < Ki : t < Kp);
            const double tv = load_or(HT, col * nc + ki + k, ok, 0.0);
            if (CDP_WORKERS * (r + 1) > 2 * CDP_TILE) {
                const int g = e - 2 * CDP_TILE, gw = g / CDH_K, gk = g % CDH_K;
                const double* src = gw == 0 ? c_inva : (gw == 1 ? c_A : (gw == 2 ? c_S : c_wtc));
                const double cv = load_or(src, ki + gk, !is_tile && g < CDP_CONST && gk < Ki, 0.0);
                treg[r] = is_tile ? tv : cv;
            } else {
                treg[r] = tv;
            }
        }
    };
    auto store_tiles = [&](int b) {
#pragma unroll
        for (int r = 0; r < CDP_TPT; ++r) {
            const int e = (tid - 64) + CDP_WORKERS * r;
            if (e < 2 * CDP_TILE) {
                const int which = e / CDP_TILE, f = e % CDP_TILE;
                (which == 0 ? Dt : St)[b * CDP_TILE + f] = treg[r];
            } else if (e < 2 * CDP_TILE + CDP_CONST) {
                cst[b * CDP_CONST + e - 2 * CDP_TILE] = treg[r];
            }
        }
    };

    for (int64_t k = tid; k < nc; k += CDP_THREADS) {
        zs[k] = 0.0;
        ds[k] = 0.0;
    }
    if (wave > 0) {
        load_tiles(0, C - 1);
        store_tiles(0);
    }
    // the chain is the critical path: let its wave win issue arbitration on its SIMD
    if (wave == 0) __builtin_amdgcn_s_setprio(3);
    if (tid == 0) {
        s_nnz[0] = 0;
        s_nnz[1] = 0;
        s_stop = 0;
    }
    lds_barrier();

    int sweeps = 0;
    double maxmu = 0.0;   // wave 0
    // thread 0's phase clocks (step application, chain, barrier wait), in LDS:
    // registers are the workers' load depth
    __shared__ long long s_tph[4];
    if (tid == 0) {
        s_tph[0] = s_tph[1] = s_tph[2] = 0;
        s_tph[3] = wall_clock64();
    }
    int64_t g = 0;
    bool done = false;
    for (int sweep = 0; sweep < max_sweeps && !done; ++sweep) {
        for (int i = 0; i < C; ++i, ++g) {
            const int b = (int)(g & 1), pb = 1 - b;   // this interval's buffers / previous steps
            const int cp = (i + C - 1) % C;            // previous chunk
            const int64_t k0 = (int64_t)i * CDH_K, kp0 = (int64_t)cp * CDH_K;
            const int K = klen(i);
            const bool have_prev = g > 0 && C > 1;
            if (wave == 0) {
                if (i == 0) maxmu = 0.0;
                const bool on = lane < K;
                const int kl = on ? (int)k0 + lane : (int)k0;
                double z = on ? zs[kl] : 0.0;
                // steps of the previous chunk onto the rows of this one
                if (have_prev && s_nnz[pb] > 0) {
                    const double* st = St + b * CDP_TILE;
                    const double* pm = mud + pb * CDH_K;
                    double a[4] = {0.0, 0.0, 0.0, 0.0};
#pragma unroll 1
                    for (int t = 0; t < CDH_K; t += 8) {
                        double sv[8], mv[8];   // all eight reads in flight before the fmas
#pragma unroll
                        for (int u = 0; u < 8; ++u) {
                            sv[u] = st[(t + u) * CDH_K + lane];
                            mv[u] = pm[t + u];
                        }
#pragma unroll
                        for (int u = 0; u < 8; ++u) a[u & 3] += sv[u] * mv[u];
                    }
                    z += on ? (a[0] + a[1]) + (a[2] + a[3]) : 0.0;
                }
                if (tid == 0) { const long long now = wall_clock64(); s_tph[0] += now - s_tph[3]; s_tph[3] = now; }
                // chain constants of this chunk (staged with its tiles; zero past K)
                const double* cb = cst + b * CDP_CONST;
                const double ia = cb[lane];
                const double d0 = on ? ds[kl] : 0.0;
                const double xl = on ? cb[CDH_K + lane] + d0 : 0.0;
                const double pv = on ? xl - (cb[2 * CDH_K + lane] - cb[3 * CDH_K + lane]) * ia : 0.0;
                const double* dt = Dt + b * CDP_TILE;
                const int K4 = (K + 3) & ~3;
                // The chain, one coordinate per step in the stored order. With
                // q = p - x, a = q - lam/a - z/a and b = q + lam/a - z/a, the step
                // mu = soft(p - z/a, lam/a) - x is the median of a, -x and b
                // (a <= b). Every lane evaluates it for its own coordinate at the
                // current z; lane t's value is step t: broadcast (two readlanes),
                // applied to every z and kept in lane t. Ten instructions a step,
                // five of them dependent.
                const double qlo = pv - xl - lam * ia, qhi = pv - xl + lam * ia, nx = -xl;
                int mlo = 0, mhi = 0;   // the steps, lane k holding step k (bits)
                double hN[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) hN[u] = dt[u * CDH_K + lane];
                for (int tt = 0; tt < K4; tt += 4) {
                    double hC[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) hC[u] = hN[u];
                    const int tn = tt + 4 < CDH_K ? tt + 4 : CDH_K - 4;   // in range; unused past K4
#pragma unroll
                    for (int u = 0; u < 4; ++u) hN[u] = dt[(tn + u) * CDH_K + lane];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        const int t = tt + u;
                        const double av = qlo - z * ia, bv = qhi - z * ia;
                        const long long own = __double_as_longlong(fmax(av, fmin(bv, nx)));
                        const int slo = __builtin_amdgcn_readlane((int)(own & 0xffffffffll), t);
                        const int shi = __builtin_amdgcn_readlane((int)(own >> 32), t);
                        const double mu =
                            __longlong_as_double(((long long)shi << 32) | (unsigned int)slo);
                        z += mu * hC[u];
                        mlo = lane == t ? slo : mlo;
                        mhi = lane == t ? shi : mhi;
                    }
                }
                const double mul = __longlong_as_double(((long long)mhi << 32) | (unsigned int)mlo);
                maxmu = fmax(maxmu, wave_max(fabs(mul)));
                if (on) {
                    zs[kl] = z;
                    ds[kl] = d0 + mul;
                }
                mud[b * CDH_K + lane] = mul;   // lanes >= K hold 0
                const bool nzs = on && mul != 0.0;
                const unsigned long long bits = __ballot(nzs);
                const int nnz = __popcll(bits);
                double* om = nzm + b * CDH_K;
                int* ol = nzl + b * CDH_K;
                if (nzs) {
                    const int pos = __popcll(bits & ((1ull << lane) - 1ull));
                    ol[pos] = lane;
                    om[pos] = mul;
                }
                const int npad = (nnz + CDP_PAD - 1) / CDP_PAD * CDP_PAD;
                if (lane >= nnz && lane < npad) {
                    ol[lane] = 0;
                    om[lane] = 0.0;
                }
                if (lane == 0) s_nnz[b] = nnz;
                if (i == C - 1) {
                    // stopping rule of the sweep: max|mu| <= tol * max|Delta|
                    double dm = 0.0;
                    for (int64_t k = lane; k < nc; k += 64) dm = fmax(dm, fabs(ds[k]));
                    dm = wave_max(dm);
                    if (lane == 0) {
                        s_stop = (maxmu <= tol * dm) ? 1 : 0;
                        stats[1] = maxmu;
                        stats[2] = dm;
                    }
                }
                if (tid == 0) { const long long now = wall_clock64(); s_tph[1] += now - s_tph[3]; s_tph[3] = now; }
            } else {
                // next interval's tiles and constants (chunk i+1 and its predecessor
                // i), issued first so that their latency hides behind the column
                // stream (with two float64 rows per thread the registers do not
                // allow it: then they follow the stream and hide behind the chain)
                constexpr bool early = ROWS == 1 || sizeof(HV) < sizeof(double);
                if (early) load_tiles((i + 1) % C, i);
                // steps of the previous chunk onto every row outside chunks cp and i
                if (have_prev && C > 2) {
                    const int np = (s_nnz[pb] + CDP_PAD - 1) / CDP_PAD * CDP_PAD;
                    const double* pm = nzm + pb * CDH_K;
                    const int* pl = nzl + pb * CDH_K;
                    const HV* hcol = HT + kp0 * nc;
                    double acc[ROWS];
                    bool rv[ROWS];
                    int rk[ROWS];
                    // worker w takes the w-th row outside the (64-aligned) chunks cp and i
                    const int64_t ea = kp0 < k0 ? kp0 : k0, eb = kp0 < k0 ? k0 : kp0;
#pragma unroll
                    for (int r = 0; r < ROWS; ++r) {
                        int64_t k = (tid - 64) + (int64_t)CDP_WORKERS * r;
                        if (k >= ea) k += CDH_K;
                        if (k >= eb) k += CDH_K;
                        rv[r] = k < nc;
                        rk[r] = rv[r] ? (int)k : 0;
                        acc[r] = 0.0;
                    }
                    // the column index is the same in every lane: a scalar base address
                    // plus a 32-bit row offset per load
                    constexpr int BATCH = CDP_PAD / ROWS;
#pragma unroll 1
                    for (int q0 = 0; q0 < np; q0 += BATCH) {
                        HV hv[ROWS][BATCH];
#pragma unroll
                        for (int q = 0; q < BATCH; ++q) {
                            const int t = __builtin_amdgcn_readfirstlane(pl[q0 + q]);
                            const HV* colp = hcol + (int64_t)t * nc;
#pragma unroll
                            for (int r = 0; r < ROWS; ++r) hv[r][q] = colp[rk[r]];
                        }
#pragma unroll
                        for (int q = 0; q < BATCH; ++q) {
                            const double m = pm[q0 + q];
#pragma unroll
                            for (int r = 0; r < ROWS; ++r) acc[r] += (double)hv[r][q] * m;
                        }
                    }
#pragma unroll
                    for (int r = 0; r < ROWS; ++r)
                        if (rv[r]) zs[rk[r]] += acc[r];
                }
                if (!early) load_tiles((i + 1) % C, i);
                store_tiles(pb);
            }
            lds_barrier();
            if (tid == 0) { const long long now = wall_clock64(); s_tph[2] += now - s_tph[3]; s_tph[3] = now; }
            if (i == C - 1) {
                ++sweeps;
                if (s_stop) {
                    done = true;
                    break;
                }
            }
        }
    }
    for (int64_t k = tid; k < nc; k += CDP_THREADS) delta[k] = ds[k];
    if (tid == 0) {
        stats[0] = (double)sweeps;
        for (int i = 0; i < 3; ++i) stats[3 + i] = (double)s_tph[i];
        stats[6] = 0.0;
    }
}

}  // namespace

// Raises a kernel's dynamic-LDS limit to the device maximum, once per kernel
// (host threads of the serving loop may launch concurrently).
static void allow_dynamic_lds(const void* kern) {
    static std::mutex mu;
    static std::vector<const void*> done;
    std::lock_guard<std::mutex> lk(mu);
    if (std::find(done.begin(), done.end(), kern) != done.end()) return;
    SIC_HIP(hipFuncSetAttribute(kern, hipFuncAttributeMaxDynamicSharedMemorySize,
                                (int)CD_MAX_LDS_BYTES));
    done.push_back(kern);
}

size_t cd_lds_bytes(int jp, bool u_in_lds) {
    const size_t fixed = (size_t)6 * CD_CHUNK + CD_CHUNK / 2 + (size_t)CD_CHUNK * CD_WPAD +
                         (size_t)CD_COLCAP + CD_COLCAP / 2 + CD_MAXB;
    return sizeof(double) * fixed + (u_in_lds ? (size_t)jp * (sizeof(double) + 1) : 0);
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
               double* ug, unsigned char* markg, double* stats, hipStream_t s) {
    prof_begin(KK_CD, s);
    const size_t lds_full = cd_lds_bytes(jp, true);
    const bool in_lds = lds_full <= CD_MAX_LDS_BYTES;
    const size_t lds = cd_lds_bytes(jp, in_lds);
    if (in_lds) {
        allow_dynamic_lds((const void*)k_cd<true>);
        hipLaunchKernelGGL(k_cd<true>, dim3(1), dim3(CD_THREADS), lds, s, jp, b, cptr, c_p, c_S,
                           c_A, c_inva, c_wtc, WJJ, lam, max_sweeps, tol, U, delta, mu_col, ug,
                           markg, stats);
    } else {
        hipLaunchKernelGGL(k_cd<false>, dim3(1), dim3(CD_THREADS), lds, s, jp, b, cptr, c_p, c_S,
                           c_A, c_inva, c_wtc, WJJ, lam, max_sweeps, tol, U, delta, mu_col, ug,
                           markg, stats);
    }
    SIC_CHECK_LAUNCH();
    // the W rows a sweep must read (one per coordinate for the model gradient)
    prof_end(KK_CD, s, 0.0, 0.0);
}

int64_t cd_hessian_limit() { return (int64_t)CDH_RMAX * CDH_THREADS; }

size_t cd_pipe_lds_bytes(int64_t ncoord) {
    return sizeof(double) * ((size_t)2 * ncoord + 4 * CDP_TILE + 4 * CDH_K + 2 * CDP_CONST) +
           sizeof(int) * 2 * CDH_K;
}

size_t cd_hessian_lds_bytes(int64_t ncoord) {
    return sizeof(double) * ((size_t)2 * ncoord + CDH_K * CDH_K + CDH_K) + sizeof(int) * CDH_K;
}

int64_t launch_cd_hessian(int64_t ncoord, int jp, const int32_t* c_p, const int32_t* c_ci,
                          const double* WJJ, const double* c_S, const double* c_A,
                          const double* c_inva, const double* c_wtc, double lam, int max_sweeps,
                          double tol, double* HT, double* delta, double* stats, hipStream_t s,
                          bool low) {
    if (ncoord <= 0) return -1;
    const size_t lds = cd_hessian_lds_bytes(ncoord);
    if (ncoord > cd_hessian_limit() || lds > CD_MAX_LDS_BYTES)
        throw SicError(SIC_EINTERNAL, "coordinate count too large for the explicit-Hessian sweep");
    const size_t lds_pipe = cd_pipe_lds_bytes(ncoord);
    // rows the workers cover: all but two chunks (all but one or none for C <= 2)
    const int prow = (int)((std::max<int64_t>(ncoord - 2 * CDH_K, 1) + CDP_WORKERS - 1) / CDP_WORKERS);
    const bool pipe = lds_pipe <= CD_MAX_LDS_BYTES && prow <= 2;
    // float storage of H (the pipelined sweep only): half the bytes the sweep streams
    const bool hf = low && pipe;
    const double hsz = hf ? 4.0 : 8.0;
    float* HTf = reinterpret_cast<float*>(HT);
    const dim3 hgrid((unsigned)((ncoord + 255) / 256), (unsigned)ncoord);
    prof_begin(KK_CD_HESS, s);
    if (hf)
        hipLaunchKernelGGL(k_cd_hess<float>, hgrid, dim3(256), 0, s, ncoord, jp, c_p, c_ci, WJJ, HTf);
    else
        hipLaunchKernelGGL(k_cd_hess<double>, hgrid, dim3(256), 0, s, ncoord, jp, c_p, c_ci, WJJ, HT);
    SIC_CHECK_LAUNCH();
    // H written once; 4 gathers of W per entry (from the L2-resident W on J')
    prof_end(KK_CD_HESS, s, hsz * (double)ncoord * ncoord, 3.0 * (double)ncoord * ncoord);
    const int rows = (int)((ncoord + CDH_THREADS - 1) / CDH_THREADS);
    auto launch = [&](auto kern) {
        allow_dynamic_lds((const void*)kern);
        prof_begin(KK_CD, s);
        hipLaunchKernelGGL(kern, dim3(1), dim3(CDH_THREADS), lds, s, ncoord, HT, c_S, c_A, c_inva,
                           c_wtc, lam, max_sweeps, tol, delta, stats);
        SIC_CHECK_LAUNCH();
    };
    auto launch_pipe = [&](auto kern, auto* H) {
        allow_dynamic_lds((const void*)kern);
        prof_begin(KK_CD, s);
        hipLaunchKernelGGL(kern, dim3(1), dim3(CDP_THREADS), lds_pipe, s, ncoord, H, c_S, c_A,
                           c_inva, c_wtc, lam, max_sweeps, tol, delta, stats);
        SIC_CHECK_LAUNCH();
    };
    if (pipe) {
        if (hf) {
            if (prow == 1) launch_pipe(k_cd_pipe<1, float>, (const float*)HTf);
            else launch_pipe(k_cd_pipe<2, float>, (const float*)HTf);
        } else {
            if (prow == 1) launch_pipe(k_cd_pipe<1, double>, (const double*)HT);
            else launch_pipe(k_cd_pipe<2, double>, (const double*)HT);
        }
    } else {
        switch (rows) {
            case 1: launch(k_cd_dense<1>); break;
            case 2: launch(k_cd_dense<2>); break;
            case 3: launch(k_cd_dense<3>); break;
            default: launch(k_cd_dense<4>); break;
        }
    }
    // one sweep streams every column of H once (hsz ncoord^2 bytes, 2 ncoord^2 flops);
    // the caller scales the record by the sweep count once it is known
    return prof_end(KK_CD, s, hsz * (double)ncoord * ncoord, 2.0 * (double)ncoord * ncoord);
}

}  // namespace sic
