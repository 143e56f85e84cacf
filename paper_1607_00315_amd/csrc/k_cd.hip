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

// HT[t * nc + k] = H[k][t] (column t of H stored contiguously).
__global__ void k_cd_hess(int64_t nc, int jp, const int32_t* __restrict__ c_p,
                          const int32_t* __restrict__ c_ci, const double* __restrict__ WJJ,
                          double* __restrict__ HT) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t t = blockIdx.y;
    if (k >= nc) return;
    const int pt = c_p[t], ct = c_ci[t];
    const int pk = c_p[k], ck = c_ci[k];
    const double* wpt = WJJ + (int64_t)pt * jp;
    const double* wct = WJJ + (int64_t)ct * jp;
    double h = wpt[pk] * wct[ck];
    if (pt != ct) h += wct[pk] * wpt[ck];
    HT[t * nc + k] = h;
}

__global__ __launch_bounds__(CDH_THREADS) void k_cd_dense(
    int64_t nc, const double* __restrict__ HT, const double* __restrict__ c_S,
    const double* __restrict__ c_A, const double* __restrict__ c_inva,
    const double* __restrict__ c_wtc, double lam, int max_sweeps, double tol,
    double* __restrict__ delta, double* __restrict__ stats) {
    extern __shared__ double sm[];
    double* zs = sm;                    // [nc] z = (W Delta W) on the coordinates
    double* ds = zs + nc;               // [nc] Delta
    double* Hc = ds + nc;               // [CDH_K][CDH_K] diagonal tile of the chunk, [t][k]
    double* mus = Hc + CDH_K * CDH_K;   // [CDH_K] steps of the chunk
    int* nzl = (int*)(mus + CDH_K);     // [CDH_K] chunk positions with a nonzero step
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
            hreg[j] = (t < K && k < K) ? HT[(k0 + t) * nc + k0 + k] : 0.0;
        }
    };
    // wave 0: the next chunk's per-coordinate constants, one coordinate per lane
    double nb_c = 0.0, nA = 0.0, ninva = 0.0;
    auto load_lane = [&](int ch) {
        const int64_t k = (int64_t)ch * CDH_K + lane;
        const bool on = k < nc;
        nb_c = on ? c_S[k] - c_wtc[k] : 0.0;
        nA = on ? c_A[k] : 0.0;
        ninva = on ? c_inva[k] : 0.0;
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
                const bool on = lane < K;
                const double bc = nb_c, inva = ninva;
                const double d0 = on ? ds[k0 + lane] : 0.0;
                const double xl = nA + d0;
                double z = on ? zs[k0 + lane] : 0.0;
                load_lane(nch);
                double mul = 0.0;
                double hn = Hc[lane];
                for (int tt = 0; tt < K; ++tt) {
                    const double h = hn;
                    if (tt + 1 < K) hn = Hc[(tt + 1) * CDH_K + lane];
                    const double x = readlane_d(xl, tt);
                    const double ia = readlane_d(inva, tt);
                    const double bb = readlane_d(bc, tt) + readlane_d(z, tt);
                    const double y = x - bb * ia;
                    const double thr = lam * ia;
                    const double sh = y > thr ? y - thr : (y < -thr ? y + thr : 0.0);
                    const double mu = sh - x;
                    z += mu * h;
                    if (lane == tt) mul = mu;
                    maxmu = fmax(maxmu, fabs(mu));
                }
                if (on) {
                    zs[k0 + lane] = z;
                    ds[k0 + lane] = d0 + mul;
                    mus[lane] = mul;
                }
                const unsigned long long nzm = __ballot(on && mul != 0.0);
                if (on && mul != 0.0)
                    nzl[__popcll(nzm & ((1ull << lane) - 1ull))] = lane;
                if (lane == 0) s_nnz = __popcll(nzm);
            }
            lds_barrier();   // steps of the chunk are in place
            if (tid == 0) { const long long now = wall_clock64(); tph[0] += now - tlast; tlast = now; }
            // z_k += sum_t H[k][t] mu_t for every coordinate outside the chunk
            const int nnz = s_nnz;
            if (nnz > 0) {
                for (int64_t k = tid; k < nc; k += CDH_THREADS) {
                    if (k >= k0 && k < k0 + K) continue;
                    const double* hk = HT + k0 * nc + k;
                    double acc = 0.0;
                    int i = 0;
                    for (; i + 8 <= nnz; i += 8) {
                        double hv[8];
#pragma unroll
                        for (int q = 0; q < 8; ++q) hv[q] = hk[(int64_t)nzl[i + q] * nc];
#pragma unroll
                        for (int q = 0; q < 8; ++q) acc += hv[q] * mus[nzl[i + q]];
                    }
                    for (; i < nnz; ++i) acc += hk[(int64_t)nzl[i] * nc] * mus[nzl[i]];
                    zs[k] += acc;
                }
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

}  // namespace

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
        static bool attr_set = false;
        if (!attr_set) {
            SIC_HIP(hipFuncSetAttribute((const void*)k_cd<true>,
                                        hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)CD_MAX_LDS_BYTES));
            attr_set = true;
        }
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

size_t cd_hessian_lds_bytes(int64_t ncoord) {
    return sizeof(double) * ((size_t)2 * ncoord + CDH_K * CDH_K + CDH_K) + sizeof(int) * CDH_K;
}

void launch_cd_hessian(int64_t ncoord, int jp, const int32_t* c_p, const int32_t* c_ci,
                       const double* WJJ, const double* c_S, const double* c_A,
                       const double* c_inva, const double* c_wtc, double lam, int max_sweeps,
                       double tol, double* HT, double* delta, double* stats, hipStream_t s) {
    if (ncoord <= 0) return;
    const size_t lds = cd_hessian_lds_bytes(ncoord);
    if (lds > CD_MAX_LDS_BYTES)
        throw SicError(SIC_EINTERNAL, "coordinate count too large for the explicit-Hessian sweep");
    prof_begin(KK_CD_HESS, s);
    hipLaunchKernelGGL(k_cd_hess, dim3((unsigned)((ncoord + 255) / 256), (unsigned)ncoord),
                       dim3(256), 0, s, ncoord, jp, c_p, c_ci, WJJ, HT);
    SIC_CHECK_LAUNCH();
    // H written once; 4 gathers of W per entry (from the L2-resident W on J')
    prof_end(KK_CD_HESS, s, 8.0 * (double)ncoord * ncoord, 3.0 * (double)ncoord * ncoord);
    static bool attr_set = false;
    if (!attr_set) {
        SIC_HIP(hipFuncSetAttribute((const void*)k_cd_dense,
                                    hipFuncAttributeMaxDynamicSharedMemorySize,
                                    (int)CD_MAX_LDS_BYTES));
        attr_set = true;
    }
    prof_begin(KK_CD, s);
    hipLaunchKernelGGL(k_cd_dense, dim3(1), dim3(CDH_THREADS), lds, s, ncoord, HT, c_S, c_A, c_inva,
                       c_wtc, lam, max_sweeps, tol, delta, stats);
    SIC_CHECK_LAUNCH();
    prof_end(KK_CD, s, 0.0, 0.0);
}

}  // namespace sic
