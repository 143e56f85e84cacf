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
        stats[7] = 0.0;
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
// xf (may be null): nxf ints cleared for the multi-workgroup sweep that follows.
template <typename HV>
__global__ void k_cd_hess(int64_t nc, int jp, const int32_t* __restrict__ c_p,
                          const int32_t* __restrict__ c_ci, const double* __restrict__ WJJ,
                          HV* __restrict__ HT, int* __restrict__ xf, int nxf) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t t = blockIdx.y;
    if (xf && blockIdx.x == 0 && blockIdx.y == 0)
        for (int e = threadIdx.x; e < nxf; e += blockDim.x) xf[e] = 0;
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
        stats[7] = 0.0;
    }
}


// Staging of the multi-workgroup sweep below: 64 x 64 tiles of H and a chunk's
// constants.
constexpr int CDP_TILE = CDH_K * CDH_K;
constexpr int CDP_CONST = 4 * CDH_K;   // a chunk's 1/a, A, S and W_rc, staged with its tiles

// ------------------------------------------------------------------------
// The same sweep over several compute units. The coordinate chain is serial,
// but applying a chunk's steps to the other coordinates' z is not, and one
// workgroup can only stream H as fast as its compute unit draws from memory
// (k_cd_dense above, about 50 GB/s). Here workgroup 0 runs the chain and helper
// workgroups 1..nhelp apply the steps. Intervals g = 0, 1, ... visit the chunks
// in order, interval g taking chunk g mod C (C chunks per sweep):
//   helpers    helper h owns the z of chunks h, h + nhelp, ... For every
//              published step list g' it adds H[own chunk][chunk g'] mu(g')
//              to that z, and after list g' it publishes the z of the chunk
//              due at interval g' + 3 (a snapshot of the steps of intervals
//              <= g' = x - 3, for x = g' + 3);
//   workgroup 0, interval g: z starts from snapshot(g), plus the steps of
//              interval g-2 on chunk g (formed by waves 1-8 during interval
//              g-1 from the tile H[chunk g][chunk g-2]), plus those of g-1
//              (accumulated by wave 0 during the chain of interval g-1 from
//              the tile H[chunk g][chunk g-1], staged with that interval's
//              tiles); wave 0 then runs the chain. Meanwhile waves 1-15 stage
//              the next interval's tiles (H[g+1][g+1] and H[g+2][g+1]) and
//              constants, waves 1-8 form the steps of interval g-1 on chunk
//              g+1, wave 9 fetches snapshot(g+1) and wave 10 publishes the
//              step list of interval g-1.
// z_k is then sum_t H[k][t] Delta_t summed by interval, and the chain and its
// visiting order are those of k_cd_dense.
//
// The lists, snapshots and their sequence flags pass through global memory as
// device-scope relaxed atomics (they bypass the per-XCD L2 caches); a writer
// waits for its data stores to complete before it stores the flag. Every wait
// gives up after two seconds and raises an abort flag that ends all
// workgroups; the host turns it into an error.
constexpr int CDM_THREADS = 1024;
constexpr int CDM_WAVES = CDM_THREADS / 64;
constexpr int CDM_HELPERS = 16;      // most helper workgroups
constexpr int CDM_OWN = 4;           // chunks per helper at most
constexpr int CDM_MAXC = CDM_HELPERS * CDM_OWN;   // chunks at most (4096 coordinates)
constexpr int CDM_RS = 128;          // step-list ring (any helper is fewer than C + 2 lists behind)
constexpr int CDM_RZ = 8;            // snapshot ring
constexpr int CDM_LAG = 3;           // snapshot(x) holds the steps of intervals <= x - 3
constexpr int CDM_PW = 8;            // waves forming the interval-(g-1) part for chunk g+1
constexpr int CDM_SNAPW = CDM_PW + 1;   // the wave fetching the snapshot
constexpr int CDM_PUBW = CDM_PW + 2;    // the wave publishing the step lists
// exchange buffer: int flags, one per 128-byte line, then the two rings (doubles)
enum { XF_PUB = 0, XF_STATUS = 32, XF_SNAP = 64 };   // snapshot flag s at XF_SNAP + 32 s
constexpr int CDM_FLAG_INTS = XF_SNAP + 32 * CDM_RZ;
constexpr int64_t CDM_XSTEPS = CDM_FLAG_INTS / 2;
constexpr int64_t CDM_XSNAP = CDM_XSTEPS + (int64_t)CDM_RS * CDH_K;
constexpr int CDM_BIG = 1 << 30;     // published-list count meaning "stop"
constexpr long long CDM_SPIN_TICKS = 200000000ll;   // two seconds of the 100 MHz clock
static_assert(CDM_RS >= CDM_MAXC + CDM_LAG, "step ring shorter than the slowest helper's lag");
static_assert(CDM_RZ >= CDM_LAG, "snapshot ring shorter than the lag");

__device__ __forceinline__ int xld_i(const int* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void xst_i(int* p, int v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double xld_d(const double* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void xst_d(double* p, double v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
// this wave's earlier memory operations complete before its later ones issue
__device__ __forceinline__ void x_drain() {
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
    __builtin_amdgcn_s_waitcnt(0);
    __atomic_signal_fence(__ATOMIC_SEQ_CST);
}

template <typename HV>
__device__ void cdm_chain(int64_t nc, const HV* __restrict__ HT, const double* __restrict__ c_S,
                          const double* __restrict__ c_A, const double* __restrict__ c_inva,
                          const double* __restrict__ c_wtc, double lam, int max_sweeps, double tol,
                          double* __restrict__ delta, double* __restrict__ stats,
                          double* __restrict__ xb, double* sm) {
    double* ds = sm;                            // [nc]
    double* Dt = ds + nc;                       // [2][64 x 64] H[chunk g][chunk g], [t][k]
    double* St = Dt + 2 * CDP_TILE;             // [2][64 x 64] H[chunk g+1][chunk g], [t][k]
    double* mud = St + 2 * CDP_TILE;            // [2][64] steps of the interval (0 past K)
    double* cst = mud + 2 * CDH_K;              // [2][4][64] the chunk's 1/a, A, S, W_rc
    double* zp = cst + 2 * CDP_CONST;           // [2][CDM_PW + 1][64] parts of the chunk's z
    int* xf = reinterpret_cast<int*>(xb);
    double* xsteps = xb + CDM_XSTEPS;
    double* xsnap = xb + CDM_XSNAP;
    __shared__ int s_nnz[2];
    __shared__ int s_stop, s_abort;
    __shared__ long long s_tph[4];
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int C = (int)((nc + CDH_K - 1) / CDH_K);
    auto klen = [&](int c) {
        const int64_t r = nc - (int64_t)c * CDH_K;
        return (int)(r < CDH_K ? r : CDH_K);
    };
    // waves 1-15: the tiles H[ci][ci] and H[cr][ci] (rows of chunk cr, the
    // one after ci) and the constants of chunk ci, into registers, then into
    // LDS buffer b
    constexpr int TPT = (2 * CDP_TILE + CDP_CONST + (CDM_THREADS - 64) - 1) / (CDM_THREADS - 64);
    double treg[TPT];
    auto load_tiles = [&](int ci, int cr) {
        const int64_t ki = (int64_t)ci * CDH_K, kr = (int64_t)cr * CDH_K;
        const int Ki = klen(ci), Kr = klen(cr);
#pragma unroll
        for (int r = 0; r < TPT; ++r) {
            const int e = (tid - 64) + (CDM_THREADS - 64) * r;
            const bool is_tile = e < 2 * CDP_TILE;
            const int which = e / CDP_TILE, f = e % CDP_TILE;
            const int t = f / CDH_K, k = f % CDH_K;
            const bool dtile = which == 0;
            // entry [t][k]: H[row k of chunk ci (Dt) or cr (St)][column t of chunk ci]
            const int64_t rbase = dtile ? ki : kr;
            const bool ok = is_tile && t < Ki && (dtile ? k < Ki : k < Kr);
            const double tv = load_or(HT, (ki + t) * nc + rbase + k, ok, 0.0);
            const int g = e - 2 * CDP_TILE, gw = g / CDH_K, gk = g % CDH_K;
            const double* src = gw == 0 ? c_inva : (gw == 1 ? c_A : (gw == 2 ? c_S : c_wtc));
            const double cv = load_or(src, ki + gk, !is_tile && g < CDP_CONST && gk < Ki, 0.0);
            treg[r] = is_tile ? tv : cv;
        }
    };
    auto store_tiles = [&](int b) {
#pragma unroll
        for (int r = 0; r < TPT; ++r) {
            const int e = (tid - 64) + (CDM_THREADS - 64) * r;
            if (e < 2 * CDP_TILE) {
                const int which = e / CDP_TILE, f = e % CDP_TILE;
                (which == 0 ? Dt : St)[b * CDP_TILE + f] = treg[r];
            } else if (e < 2 * CDP_TILE + CDP_CONST) {
                cst[b * CDP_CONST + e - 2 * CDP_TILE] = treg[r];
            }
        }
    };

    for (int64_t k = tid; k < nc; k += CDM_THREADS) ds[k] = 0.0;
    for (int e = tid; e < 2 * (CDM_PW + 1) * CDH_K; e += CDM_THREADS) zp[e] = 0.0;
    if (wave > 0) {
        load_tiles(0, 1 % C);
        store_tiles(0);
    }
    if (wave == 0) __builtin_amdgcn_s_setprio(3);   // the chain is the critical path
    if (tid == 0) {
        s_nnz[0] = s_nnz[1] = 0;
        s_stop = 0;
        s_abort = 0;
        s_tph[0] = s_tph[1] = s_tph[2] = 0;
        s_tph[3] = wall_clock64();
    }
    lds_barrier();

    int sweeps = 0;
    double maxmu = 0.0;   // wave 0
    double zcarry = 0.0;  // wave 0: the steps of the last chain on the rows of the next chunk
    int64_t g = 0;
    bool done = false;
    for (int sweep = 0; sweep < max_sweeps && !done; ++sweep) {
        for (int i = 0; i < C; ++i, ++g) {
            const int b = (int)(g & 1), pb = 1 - b;
            const int K = klen(i);
            if (wave == 0) {
                if (i == 0) maxmu = 0.0;
                const bool on = lane < K;
                const int kl = on ? i * CDH_K + lane : i * CDH_K;
                // z: the steps of interval g-1 (accumulated during its chain), the
                // snapshot, then the parts of interval g-2 in wave order
                const double* zb = zp + b * (CDM_PW + 1) * CDH_K;
                double z = zcarry + zb[CDM_PW * CDH_K + lane];
#pragma unroll
                for (int w = 0; w < CDM_PW; ++w) z += zb[w * CDH_K + lane];
                z = on ? z : 0.0;
                if (tid == 0) { const long long now = wall_clock64(); s_tph[0] += now - s_tph[3]; s_tph[3] = now; }
                const double* cb = cst + b * CDP_CONST;
                const double ia = cb[lane];
                const double d0 = on ? ds[kl] : 0.0;
                const double xl = on ? cb[CDH_K + lane] + d0 : 0.0;
                const double pv = on ? xl - (cb[2 * CDH_K + lane] - cb[3 * CDH_K + lane]) * ia : 0.0;
                const double* dt = Dt + b * CDP_TILE;
                const double* sn = St + b * CDP_TILE;
                const int K4 = (K + 3) & ~3;
                // The chain, one coordinate per step in the stored order. With
                // q = p - x, a = q - lam/a - z/a and b = q + lam/a - z/a, the step
                // mu = soft(p - z/a, lam/a) - x is the median of a, -x and b
                // (a <= b). Every lane evaluates it for its own coordinate at the
                // current z; lane t's value is step t: broadcast (two readlanes),
                // applied to every z and kept in lane t. The same step goes into
                // zn, the next chunk's rows (tile H[next][this]), off the chain's
                // dependency path: the next interval starts from it.
                const double qlo = pv - xl - lam * ia, qhi = pv - xl + lam * ia, nx = -xl;
                int mlo = 0, mhi = 0;
                double zn = 0.0;
                double hN[4], sN[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    hN[u] = dt[u * CDH_K + lane];
                    sN[u] = sn[u * CDH_K + lane];
                }
                for (int tt = 0; tt < K4; tt += 4) {
                    double hC[4], sC[4];
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        hC[u] = hN[u];
                        sC[u] = sN[u];
                    }
                    const int tn = tt + 4 < CDH_K ? tt + 4 : CDH_K - 4;
#pragma unroll
                    for (int u = 0; u < 4; ++u) {
                        hN[u] = dt[(tn + u) * CDH_K + lane];
                        sN[u] = sn[(tn + u) * CDH_K + lane];
                    }
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
                        zn += mu * sC[u];
                        mlo = lane == t ? slo : mlo;
                        mhi = lane == t ? shi : mhi;
                    }
                }
                zcarry = zn;
                double mul = __longlong_as_double(((long long)mhi << 32) | (unsigned int)mlo);
                mul = on ? mul : 0.0;
                maxmu = fmax(maxmu, wave_max(fabs(mul)));
                if (on) ds[kl] = d0 + mul;
                mud[b * CDH_K + lane] = mul;
                const int nnz = __popcll(__ballot(mul != 0.0));
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
                const int cn = (i + 1) % C;                  // the next interval's chunk
                load_tiles(cn, (i + 2) % C);
                double* zn = zp + pb * (CDM_PW + 1) * CDH_K;
                if (wave <= CDM_PW) {
                    // steps of interval g-1 on the rows of chunk cn: tile rows t of
                    // this wave's eighth of chunk g-1
                    double acc = 0.0;
                    if (g > 0 && s_nnz[b ^ 1] > 0) {
                        const int cq = (int)((g - 1) % C);
                        const int Kq = klen(cq), Kn = klen(cn);
                        const int t0 = (wave - 1) * (CDH_K / CDM_PW);
                        const double* pm = mud + pb * CDH_K;
                        double hv[CDH_K / CDM_PW];
#pragma unroll
                        for (int u = 0; u < CDH_K / CDM_PW; ++u) {
                            const int t = t0 + u;
                            hv[u] = load_or(HT, ((int64_t)cq * CDH_K + t) * nc + (int64_t)cn * CDH_K + lane,
                                            t < Kq && lane < Kn, 0.0);
                        }
#pragma unroll
                        for (int u = 0; u < CDH_K / CDM_PW; ++u) acc += hv[u] * pm[t0 + u];
                    }
                    zn[(wave - 1) * CDH_K + lane] = acc;
                } else if (wave == CDM_PUBW) {
                    // publish the list of interval g-1 (wave 0 does not wait on global stores)
                    if (g > 0) {
                        xst_d(xsteps + ((g - 1) % CDM_RS) * CDH_K + lane, mud[pb * CDH_K + lane]);
                        x_drain();
                        if (lane == 0) xst_i(xf + XF_PUB, (int)g);
                    }
                } else if (wave == CDM_SNAPW) {
                    // snapshot(g+1) from the helper that owns chunk cn
                    double v = 0.0;
                    if (g + 1 >= CDM_LAG) {
                        const int slot = (int)((g + 1) % CDM_RZ);
                        const long long t0 = wall_clock64();
                        int polls = 0;
                        bool ok = true;
                        while (xld_i(xf + XF_SNAP + 32 * slot) != (int)(g + 1)) {
                            if ((++polls & 15) == 0) {
                                if (xld_i(xf + XF_STATUS) == 2 || wall_clock64() - t0 > CDM_SPIN_TICKS) {
                                    ok = false;
                                    break;
                                }
                            }
                            __builtin_amdgcn_s_sleep(1);
                        }
                        __atomic_signal_fence(__ATOMIC_SEQ_CST);
                        if (ok) v = xld_d(xsnap + (int64_t)slot * CDH_K + lane);
                        else if (lane == 0) s_abort = 1;
                    }
                    zn[CDM_PW * CDH_K + lane] = v;
                }
                store_tiles(pb);
            }
            lds_barrier();
            if (tid == 0) { const long long now = wall_clock64(); s_tph[2] += now - s_tph[3]; s_tph[3] = now; }
            if (s_abort) {
                done = true;
                break;
            }
            if (i == C - 1) {
                ++sweeps;
                if (s_stop) {
                    done = true;
                    break;
                }
            }
        }
    }
    // the helpers stop at the next list they wait for
    if (tid == 0) {
        x_drain();
        xst_i(xf + XF_STATUS, s_abort ? 2 : 1);
        x_drain();
        xst_i(xf + XF_PUB, CDM_BIG);
    }
    for (int64_t k = tid; k < nc; k += CDM_THREADS) delta[k] = ds[k];
    if (tid == 0) {
        stats[0] = (double)sweeps;
        for (int i = 0; i < 3; ++i) stats[3 + i] = (double)s_tph[i];
        stats[6] = 0.0;
        stats[7] = s_abort ? 1.0 : 0.0;
    }
}

template <typename HV>
__device__ void cdm_helper(int64_t nc, const HV* __restrict__ HT, int nhelp,
                           double* __restrict__ xb, double* sm) {
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int h = (int)blockIdx.x - 1;
    const int C = (int)((nc + CDH_K - 1) / CDH_K);
    const int nown = (C - h + nhelp - 1) / nhelp;   // chunks h, h + nhelp, ...
    double* part = sm;                               // [2][CDM_OWN][16][64]
    double* mus = part + 2 * CDM_OWN * CDM_WAVES * CDH_K;   // [2][64]
    int* xf = reinterpret_cast<int*>(xb);
    const double* xsteps = xb + CDM_XSTEPS;
    double* xsnap = xb + CDM_XSNAP;
    __shared__ int s_exit;
    auto klen = [&](int c) {
        const int64_t r = nc - (int64_t)c * CDH_K;
        return (int)(r < CDH_K ? r : CDH_K);
    };
    // this thread's tile entries of list gg: rows t = wave + 16 r of chunk
    // gg mod C, column `lane` of each owned chunk
    double tcur[CDM_OWN][4], tnext[CDM_OWN][4];
    auto load = [&](int64_t gg, double (&tv)[CDM_OWN][4]) {
        const int c = (int)(gg % C);
        const int Kc = klen(c);
#pragma unroll
        for (int o = 0; o < CDM_OWN; ++o) {
            const int j = h + o * nhelp;
            const bool oj = o < nown;
            const int Kj = oj ? klen(j) : 0;
#pragma unroll
            for (int r = 0; r < 4; ++r) {
                const int t = wave + CDM_WAVES * r;
                tv[o][r] = load_or(HT, ((int64_t)c * CDH_K + t) * nc + (int64_t)j * CDH_K + lane,
                                   oj && t < Kc && lane < Kj, 0.0);
            }
        }
    };
    double zown[CDM_OWN];   // wave 0: z of the owned chunks, lane k = row k
#pragma unroll
    for (int o = 0; o < CDM_OWN; ++o) zown[o] = 0.0;
    if (tid == 0) s_exit = 0;
    load(0, tcur);
    for (int64_t gg = 0;; ++gg) {
        const int q = (int)(gg & 1);
        if (wave == 0) {
            // wait for list gg, then fetch it
            const long long t0 = wall_clock64();
            int polls = 0, pub;
            while ((pub = xld_i(xf + XF_PUB)) <= (int)gg) {
                if ((++polls & 15) == 0 && wall_clock64() - t0 > CDM_SPIN_TICKS) {
                    pub = -1;
                    break;
                }
                __builtin_amdgcn_s_sleep(1);
            }
            __atomic_signal_fence(__ATOMIC_SEQ_CST);
            if (pub < 0 || pub >= CDM_BIG) {
                if (pub < 0 && lane == 0) xst_i(xf + XF_STATUS, 2);
                if (lane == 0) s_exit = 1;
            } else {
                mus[q * CDH_K + lane] = xld_d(xsteps + (gg % CDM_RS) * CDH_K + lane);
            }
        }
        lds_barrier();
        if (s_exit) break;
        load(gg + 1, tnext);
        double m[4];
#pragma unroll
        for (int r = 0; r < 4; ++r) m[r] = mus[q * CDH_K + wave + CDM_WAVES * r];
#pragma unroll
        for (int o = 0; o < CDM_OWN; ++o) {
            if (o < nown) {
                const double a = (tcur[o][0] * m[0] + tcur[o][1] * m[1]) +
                                 (tcur[o][2] * m[2] + tcur[o][3] * m[3]);
                part[((q * CDM_OWN + o) * CDM_WAVES + wave) * CDH_K + lane] = a;
            }
        }
        lds_barrier();
        if (wave == 0) {
            // the owned chunk due at interval gg + 3 gets its snapshot
            const int due = (int)((gg + CDM_LAG) % C);
#pragma unroll
            for (int o = 0; o < CDM_OWN; ++o) {
                if (o < nown) {
                    const double* pp = part + (q * CDM_OWN + o) * CDM_WAVES * CDH_K;
                    double s = 0.0;
#pragma unroll
                    for (int w = 0; w < CDM_WAVES; ++w) s += pp[w * CDH_K + lane];
                    zown[o] += s;
                    if (h + o * nhelp == due) {
                        const int slot = (int)((gg + CDM_LAG) % CDM_RZ);
                        xst_d(xsnap + (int64_t)slot * CDH_K + lane, zown[o]);
                        x_drain();
                        if (lane == 0) xst_i(xf + XF_SNAP + 32 * slot, (int)(gg + CDM_LAG));
                    }
                }
            }
        }
#pragma unroll
        for (int o = 0; o < CDM_OWN; ++o)
#pragma unroll
            for (int r = 0; r < 4; ++r) tcur[o][r] = tnext[o][r];
    }
}

template <typename HV>
__global__ __launch_bounds__(CDM_THREADS) void k_cd_multi(
    int64_t nc, const HV* __restrict__ HT, const double* __restrict__ c_S,
    const double* __restrict__ c_A, const double* __restrict__ c_inva,
    const double* __restrict__ c_wtc, double lam, int max_sweeps, double tol,
    double* __restrict__ delta, double* __restrict__ stats, double* __restrict__ xb, int nhelp) {
    extern __shared__ double sm[];
    if (blockIdx.x == 0)
        cdm_chain<HV>(nc, HT, c_S, c_A, c_inva, c_wtc, lam, max_sweeps, tol, delta, stats, xb, sm);
    else
        cdm_helper<HV>(nc, HT, nhelp, xb, sm);
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

size_t cd_multi_lds_bytes(int64_t ncoord) {
    const size_t chain = sizeof(double) * ((size_t)ncoord + 4 * CDP_TILE + 2 * CDH_K + 2 * CDP_CONST +
                                           2 * (CDM_PW + 1) * CDH_K);
    const size_t helper = sizeof(double) * ((size_t)2 * CDM_OWN * CDM_WAVES * CDH_K + 2 * CDH_K);
    return std::max(chain, helper);
}

size_t cd_exchange_doubles() { return (size_t)CDM_XSNAP + (size_t)CDM_RZ * CDH_K; }

size_t cd_hessian_lds_bytes(int64_t ncoord) {
    return sizeof(double) * ((size_t)2 * ncoord + CDH_K * CDH_K + CDH_K) + sizeof(int) * CDH_K;
}

int64_t launch_cd_hessian(int64_t ncoord, int jp, const int32_t* c_p, const int32_t* c_ci,
                          const double* WJJ, const double* c_S, const double* c_A,
                          const double* c_inva, const double* c_wtc, double lam, int max_sweeps,
                          double tol, double* HT, double* delta, double* stats, double* xbuf,
                          hipStream_t s, bool low) {
    if (ncoord <= 0) return -1;
    const size_t lds = cd_hessian_lds_bytes(ncoord);
    if (ncoord > cd_hessian_limit() || lds > CD_MAX_LDS_BYTES)
        throw SicError(SIC_EINTERNAL, "coordinate count too large for the explicit-Hessian sweep");
    const int C = (int)((ncoord + CDH_K - 1) / CDH_K);
    const size_t lds_multi = cd_multi_lds_bytes(ncoord);
    const bool multi = xbuf && C <= CDM_MAXC && lds_multi <= CD_MAX_LDS_BYTES;
    // float storage of H (the multi-workgroup sweep only): half the bytes the sweep streams
    const bool hf = low && multi;
    const double hsz = hf ? 4.0 : 8.0;
    float* HTf = reinterpret_cast<float*>(HT);
    int* xf = multi ? reinterpret_cast<int*>(xbuf) : nullptr;
    const dim3 hgrid((unsigned)((ncoord + 255) / 256), (unsigned)ncoord);
    prof_begin(KK_CD_HESS, s);
    if (hf)
        hipLaunchKernelGGL(k_cd_hess<float>, hgrid, dim3(256), 0, s, ncoord, jp, c_p, c_ci, WJJ, HTf,
                           xf, CDM_FLAG_INTS);
    else
        hipLaunchKernelGGL(k_cd_hess<double>, hgrid, dim3(256), 0, s, ncoord, jp, c_p, c_ci, WJJ, HT,
                           xf, CDM_FLAG_INTS);
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
    auto launch_multi = [&](auto kern, auto* H) {
        allow_dynamic_lds((const void*)kern);
        const int nhelp = std::min(C, CDM_HELPERS);
        prof_begin(KK_CD, s);
        hipLaunchKernelGGL(kern, dim3(1 + nhelp), dim3(CDM_THREADS), lds_multi, s, ncoord, H, c_S,
                           c_A, c_inva, c_wtc, lam, max_sweeps, tol, delta, stats, xbuf, nhelp);
        SIC_CHECK_LAUNCH();
    };
    if (multi) {
        if (hf) launch_multi(k_cd_multi<float>, (const float*)HTf);
        else launch_multi(k_cd_multi<double>, (const double*)HT);
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
