// Gradient, free-set screening, neighbourhood and working-set gathers of one
// block update (Section 5.2 eq. (active_set), Section 6.1 eq. (active_set_j),
// eq. (extended_set); Section 7 eq. (MLE_l1_prior_C) at coarse levels).
//
// Layout of a block I = [j0, j0+b): every dense n x b array (S_J, W_I, A_J)
// is row-major, so a workgroup thread owns one block column and consecutive
// threads read consecutive addresses of a row.  The free set is emitted in
// column-major order (column c ascending, row r ascending), both triangles of
// the in-block part included; the descent coordinates are the subset with
// r outside I or r <= c.
#include "profiler.h"

namespace sic {

namespace {

__device__ inline double sgn(double a) { return a > 0.0 ? 1.0 : -1.0; }

// min-norm subgradient entry (Section 4, eq. (subgradient1))
__device__ inline double mnorm(double g, double a, double lam) {
    return a != 0.0 ? fabs(g + lam * sgn(a)) : fmax(fabs(g) - lam, 0.0);
}

__global__ void k_scatter_aj(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                             const double* __restrict__ val, int64_t j0, int b,
                             double* __restrict__ AJ) {
    const int ci = blockIdx.x;
    const int64_t c = j0 + ci;
    for (int64_t e = rowptr[c] + threadIdx.x; e < rowptr[c + 1]; e += blockDim.x)
        AJ[(int64_t)col[e] * b + ci] = val[e];
}

// Fine level: all n rows of every block column are candidates.
// pass 0: per-(tile, column) counts, neighbour flags, KKT partials
// pass 1: compacted entries at offsets from the column-major scan
__global__ __launch_bounds__(256) void k_screen_fine(
    int pass, int64_t n, int64_t j0, int b, int rows_per_tile, double lam,
    const double* __restrict__ SJ, const double* __restrict__ WI, const double* __restrict__ AJ,
    int32_t* __restrict__ tilecount, const int32_t* __restrict__ offsets,
    int32_t* __restrict__ e_row, double* __restrict__ e_g, double* __restrict__ e_s,
    double* __restrict__ e_a, double* __restrict__ e_w, int32_t* __restrict__ nflag,
    double* __restrict__ kkt) {
    const int ci = threadIdx.x;
    const int tile = blockIdx.x;
    const int64_t r0 = (int64_t)tile * rows_per_tile;
    const int64_t r1 = r0 + rows_per_tile < n ? r0 + rows_per_tile : n;
    const int64_t c = j0 + ci;
    int cnt = 0;
    double kmax = 0.0, ksum = 0.0;
    if (ci < b) {
        int pos = pass ? offsets[tile * b + ci] : 0;
        // rows in groups of sixteen: all 48 loads in flight before the (ordered)
        // screening of the group; rows past the tile end load row r0 and are skipped
        constexpr int G = 16;
        for (int64_t rg = r0; rg < r1; rg += G) {
            double sv[G], wv[G], av[G];
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int64_t r = rg + u < r1 ? rg + u : r0;
                const int64_t o = r * b + ci;
                sv[u] = SJ[o];
                wv[u] = WI ? WI[o] : (r == c ? 1.0 : 0.0);
                av[u] = AJ[o];
            }
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int64_t r = rg + u;
                if (r < r1) {   // rows past the tile end were loaded as row r0
                    const double s = sv[u];
                    const double w = wv[u];
                    const double a = av[u];
                    const double g = s - w;
                    const bool fr = (a != 0.0) || (fabs(g) > lam);
                    if (pass == 0) {
                        const double mv = mnorm(g, a, lam);
                        kmax = fmax(kmax, mv);
                        ksum += mv;
                        if (fr && (r < j0 || r >= j0 + b)) nflag[r] = 1;
                    } else if (fr) {
                        e_row[pos] = (int32_t)r;
                        e_g[pos] = g;
                        e_s[pos] = s;
                        e_a[pos] = a;
                        e_w[pos] = w;
                        ++pos;
                    }
                    cnt += fr ? 1 : 0;
                }
            }
        }
        if (pass == 0) tilecount[tile * b + ci] = cnt;
    }
    if (pass == 0) {
        __shared__ double smax[256], ssum[256];
        smax[threadIdx.x] = kmax;
        ssum[threadIdx.x] = ksum;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) {
                smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + off]);
                ssum[threadIdx.x] += ssum[threadIdx.x + off];
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) {
            kkt[2 * tile + 0] = smax[0];
            kkt[2 * tile + 1] = ssum[0];
        }
    }
}

// Combine per-tile KKT partials into the sweep accumulators (fixed order).
__global__ void k_kkt_accumulate(const double* __restrict__ kkt, int tiles, double* __restrict__ acc) {
    if (threadIdx.x != 0) return;
    double m = acc[0], s = 0.0;
    for (int t = 0; t < tiles; ++t) {
        m = fmax(m, kkt[2 * t]);
        s += kkt[2 * t + 1];
    }
    acc[0] = m;
    acc[1] += s;
}

// Neighbourhood N and the local index map of J' = I u N (I first, then N ascending).
__global__ void k_nbr_compact(const int32_t* __restrict__ flag, const int64_t* __restrict__ scan,
                              int64_t n, int64_t j0, int b, int32_t* __restrict__ Jp,
                              int32_t* __restrict__ lmap) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    if (r >= j0 && r < j0 + b) {
        lmap[r] = (int32_t)(r - j0);
        Jp[r - j0] = (int32_t)r;
    } else if (flag[r]) {
        const int64_t pos = scan[r];
        lmap[r] = (int32_t)(b + pos);
        Jp[b + pos] = (int32_t)r;
    }
}

// Compaction of flagged rows into a list plus a row -> position map (no I offset).
__global__ void k_flag_compact(const int32_t* __restrict__ flag, const int64_t* __restrict__ scan,
                               int64_t n, int32_t* __restrict__ list, int32_t* __restrict__ map) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n || !flag[r]) return;
    const int64_t pos = scan[r];
    list[pos] = (int32_t)r;
    map[r] = (int32_t)pos;
}

// Reset flags and maps of the rows in a list (plus the block rows for lmap).
__global__ void k_reset_rows(const int32_t* __restrict__ list, int64_t count,
                             int32_t* __restrict__ flag, int32_t* __restrict__ map) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const int32_t r = list[t];
    if (flag) flag[r] = 0;
    if (map) map[r] = -1;
}

// Coordinates: per column, the free entries with r outside I or r <= c.
__global__ __launch_bounds__(64) void k_coord_count(const int64_t* __restrict__ colptr,
                                                    const int32_t* __restrict__ e_row, int64_t j0,
                                                    int b, int32_t* __restrict__ ccount) {
    const int ci = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t c = j0 + ci;
    int cnt = 0;
    for (int64_t e = colptr[ci] + lane; e < colptr[ci + 1]; e += 64) {
        const int64_t r = e_row[e];
        cnt += (r < j0 || r >= j0 + b || r <= c) ? 1 : 0;
    }
    for (int off = 32; off > 0; off >>= 1) cnt += __shfl_xor(cnt, off, 64);
    if (lane == 0) ccount[ci] = cnt;
}

__global__ __launch_bounds__(64) void k_coord_fill(
    const int64_t* __restrict__ colptr, const int32_t* __restrict__ e_row,
    const double* __restrict__ e_s, const double* __restrict__ e_a,
    const int64_t* __restrict__ cptr, const int32_t* __restrict__ lmap, int64_t j0, int b,
    int32_t* __restrict__ c_p, int32_t* __restrict__ c_e, double* __restrict__ c_S,
    double* __restrict__ c_A) {
    const int ci = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t c = j0 + ci;
    int64_t out = cptr[ci];
    for (int64_t e0 = colptr[ci]; e0 < colptr[ci + 1]; e0 += 64) {
        const int64_t e = e0 + lane;
        bool pred = false;
        int64_t r = 0;
        if (e < colptr[ci + 1]) {
            r = e_row[e];
            pred = (r < j0 || r >= j0 + b || r <= c);
        }
        const unsigned long long mask = __ballot(pred);
        const int pre = __popcll(mask & ((1ull << lane) - 1ull));
        if (pred) {
            const int64_t t = out + pre;
            c_p[t] = lmap[r];
            c_e[t] = (int32_t)e;
            c_S[t] = e_s[e];
            c_A[t] = e_a[e];
        }
        out += __popcll(mask);
    }
}

// W restricted to J' x J' (row-major jp x jp), symmetrised where two sources exist.
// mode 0 (finest level): WI = W[:, I] (n x b), WN = W[:, N] (n x nN)
// mode 1 (coarse level): WII (b x b), WNC = W[:, N^C] (n x nC), cmap: row -> column of WNC
__global__ __launch_bounds__(256) void k_gather_wjj(
    int mode, const int32_t* __restrict__ Jp, int jp, int b, const double* __restrict__ WI,
    const double* __restrict__ WN, int64_t nN, const double* __restrict__ WII,
    const double* __restrict__ WNC, int64_t nC, const int32_t* __restrict__ cmap,
    double* __restrict__ WJJ) {
    const int p = blockIdx.x;
    const int64_t gp = Jp[p];
    for (int q = threadIdx.x; q < jp; q += blockDim.x) {
    const int64_t gq = Jp[q];
    double v;
    if (mode == 0) {
        if (p < b && q < b)
            v = 0.5 * (WI[gp * b + q] + WI[gq * b + p]);
        else if (q < b)
            v = WI[gp * b + q];
        else if (p < b)
            v = WI[gq * b + p];
        else
            v = 0.5 * (WN[gp * nN + (q - b)] + WN[gq * nN + (p - b)]);
    } else {
        if (p < b && q < b)
            v = 0.5 * (WII[(int64_t)p * b + q] + WII[(int64_t)q * b + p]);
        else if (q < b)
            v = WNC[gq * nC + cmap[gp]];
        else if (p < b)
            v = WNC[gp * nC + cmap[gq]];
        else
            v = 0.5 * (WNC[gp * nC + cmap[gq]] + WNC[gq * nC + cmap[gp]]);
    }
    WJJ[(int64_t)p * jp + q] = v;
    }
}

// ---------------------------------------------------------------- coarse levels

// Column index of every candidate entry of the block columns (C_l rows j0..j0+b-1).
__global__ void k_expand_cand(const int64_t* __restrict__ crow, int64_t j0, int64_t base,
                              int32_t* __restrict__ cand_col) {
    const int ci = blockIdx.x;
    const int64_t c = j0 + ci;
    for (int64_t e = crow[c] + threadIdx.x; e < crow[c + 1]; e += blockDim.x)
        cand_col[e - base] = (int32_t)c;
}

__global__ void k_flag_cand(const int32_t* __restrict__ ccol, int64_t base, int64_t count,
                            int64_t j0, int b, int32_t* __restrict__ flag) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const int64_t r = ccol[base + t];
    if (r < j0 || r >= j0 + b) flag[r] = 1;
}

// K = A_{I, N^C} W_{N^C, I} (App. A.2, eq. (reducingGradients1)); K is b x b row-major.
// W_{q, j} for q in N^C is read from the solved columns: WNC[(j0 + j) * nC + cmap[q]].
__global__ void k_a2_k(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                       const double* __restrict__ val, int64_t j0, int b,
                       const double* __restrict__ WNC, int64_t nC, const int32_t* __restrict__ cmap,
                       double* __restrict__ K, int32_t* __restrict__ err) {
    const int i = blockIdx.x;
    const int j = threadIdx.x;
    if (j >= b) return;
    double s = 0.0;
    for (int64_t e = rowptr[j0 + i]; e < rowptr[j0 + i + 1]; ++e) {
        const int64_t q = col[e];
        if (q >= j0 && q < j0 + b) continue;
        const int32_t cq = cmap[q];
        if (cq < 0) {
            *err = 1;   // support outside C_l: violates supp(A) in C_l
            continue;
        }
        s += val[e] * WNC[(j0 + j) * nC + cq];
    }
    K[(int64_t)i * b + j] = s;
}

// Dense A_II (b x b) from the CSR rows of the block.
__global__ void k_dense_aii(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                            const double* __restrict__ val, int64_t j0, int b,
                            double* __restrict__ out) {
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < b; j += blockDim.x) out[(int64_t)i * b + j] = 0.0;
    __syncthreads();
    for (int64_t e = rowptr[j0 + i] + threadIdx.x; e < rowptr[j0 + i + 1]; e += blockDim.x) {
        const int64_t q = col[e];
        if (q >= j0 && q < j0 + b) out[(int64_t)i * b + (q - j0)] = val[e];
    }
}

// Coarse screening: candidates of column c are the C_l entries of row c.
// pass 0 counts per column and flags neighbour rows, pass 1 fills in order.
__global__ __launch_bounds__(64) void k_screen_coarse(
    int pass, const int64_t* __restrict__ crow, const int32_t* __restrict__ ccol, int64_t base,
    int64_t j0, int b, double lam, const double* __restrict__ S_cand,
    const double* __restrict__ WII, const double* __restrict__ WNC, int64_t nC,
    const int32_t* __restrict__ cmap, const double* __restrict__ AJ,
    int32_t* __restrict__ ccount, const int64_t* __restrict__ colptr,
    int32_t* __restrict__ e_row, double* __restrict__ e_g, double* __restrict__ e_s,
    double* __restrict__ e_a, double* __restrict__ e_w, int32_t* __restrict__ nflag) {
    const int ci = blockIdx.x;
    const int lane = threadIdx.x;
    const int64_t c = j0 + ci;
    int64_t out = pass ? colptr[ci] : 0;
    int cnt = 0;
    for (int64_t e0 = crow[c]; e0 < crow[c + 1]; e0 += 64) {
        const int64_t e = e0 + lane;
        bool fr = false;
        int64_t r = 0;
        double g = 0.0, s = 0.0, a = 0.0, w = 0.0;
        if (e < crow[c + 1]) {
            r = ccol[e];
            s = S_cand[e - base];
            const bool inI = r >= j0 && r < j0 + b;
            w = inI ? WII[(r - j0) * b + ci] : WNC[c * nC + cmap[r]];
            a = AJ[r * b + ci];
            g = s - w;
            fr = (a != 0.0) || (fabs(g) > lam);
            if (pass == 0 && fr && !inI) nflag[r] = 1;
        }
        const unsigned long long mask = __ballot(fr);
        if (pass == 1 && fr) {
            const int64_t t = out + __popcll(mask & ((1ull << lane) - 1ull));
            e_row[t] = (int32_t)r;
            e_g[t] = g;
            e_s[t] = s;
            e_a[t] = a;
            e_w[t] = w;
        }
        out += __popcll(mask);
        cnt += __popcll(mask);
    }
    if (pass == 0 && lane == 0) ccount[ci] = cnt;
}

}  // namespace

void launch_scatter_aj(const DevCSR& A, int64_t j0, int b, double* AJ, hipStream_t s) {
    hipLaunchKernelGGL(k_scatter_aj, dim3(b), dim3(64), 0, s, A.rowptr.p, A.col.p, A.val.p, j0, b, AJ);
    SIC_CHECK_LAUNCH();
}

void launch_screen_fine(int pass, int64_t n, int64_t j0, int b, int rows_per_tile, int tiles,
                        double lam, const double* SJ, const double* WI, const double* AJ,
                        int32_t* tilecount, const int32_t* offsets, int32_t* e_row, double* e_g,
                        double* e_s, double* e_a, double* e_w, int32_t* nflag, double* kkt,
                        hipStream_t s) {
    prof_begin(KK_SCREEN, s);
    hipLaunchKernelGGL(k_screen_fine, dim3(tiles), dim3(256), 0, s, pass, n, j0, b, rows_per_tile,
                       lam, SJ, WI, AJ, tilecount, offsets, e_row, e_g, e_s, e_a, e_w, nflag, kkt);
    SIC_CHECK_LAUNCH();
    // algorithmic: S_J, W_I (when present) and A_J read once
    prof_end(KK_SCREEN, s, (double)n * b * 8.0 * (WI ? 3.0 : 2.0), 4.0 * (double)n * b);
}

void launch_kkt_accumulate(const double* kkt, int tiles, double* acc, hipStream_t s) {
    hipLaunchKernelGGL(k_kkt_accumulate, dim3(1), dim3(64), 0, s, kkt, tiles, acc);
    SIC_CHECK_LAUNCH();
}

void launch_nbr_compact(const int32_t* flag, const int64_t* scan, int64_t n, int64_t j0, int b,
                        int32_t* Jp, int32_t* lmap, hipStream_t s) {
    hipLaunchKernelGGL(k_nbr_compact, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, flag, scan,
                       n, j0, b, Jp, lmap);
    SIC_CHECK_LAUNCH();
}

void launch_flag_compact(const int32_t* flag, const int64_t* scan, int64_t n, int32_t* list,
                         int32_t* map, hipStream_t s) {
    hipLaunchKernelGGL(k_flag_compact, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, flag,
                       scan, n, list, map);
    SIC_CHECK_LAUNCH();
}

void launch_reset_rows(const int32_t* list, int64_t count, int32_t* flag, int32_t* map, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_reset_rows, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, list,
                       count, flag, map);
    SIC_CHECK_LAUNCH();
}

void launch_coord_count(const int64_t* colptr, const int32_t* e_row, int64_t j0, int b,
                        int32_t* ccount, hipStream_t s) {
    hipLaunchKernelGGL(k_coord_count, dim3(b), dim3(64), 0, s, colptr, e_row, j0, b, ccount);
    SIC_CHECK_LAUNCH();
}

void launch_coord_fill(const int64_t* colptr, const int32_t* e_row, const double* e_s,
                       const double* e_a, const int64_t* cptr, const int32_t* lmap, int64_t j0,
                       int b, int32_t* c_p, int32_t* c_e, double* c_S, double* c_A, hipStream_t s) {
    hipLaunchKernelGGL(k_coord_fill, dim3(b), dim3(64), 0, s, colptr, e_row, e_s, e_a, cptr, lmap,
                       j0, b, c_p, c_e, c_S, c_A);
    SIC_CHECK_LAUNCH();
}

void launch_gather_wjj(int mode, const int32_t* Jp, int jp, int b, const double* WI,
                       const double* WN, int64_t nN, const double* WII, const double* WNC,
                       int64_t nC, const int32_t* cmap, double* WJJ, hipStream_t s) {
    if (jp <= 0) return;
    hipLaunchKernelGGL(k_gather_wjj, dim3((unsigned)jp), dim3(256), 0, s, mode, Jp, jp, b, WI, WN, nN, WII, WNC,
                       nC, cmap, WJJ);
    SIC_CHECK_LAUNCH();
}

void launch_expand_cand(const int64_t* crow, int64_t j0, int b, int64_t base, int32_t* cand_col,
                        hipStream_t s) {
    hipLaunchKernelGGL(k_expand_cand, dim3(b), dim3(64), 0, s, crow, j0, base, cand_col);
    SIC_CHECK_LAUNCH();
}

void launch_flag_cand(const int32_t* ccol, int64_t base, int64_t count, int64_t j0, int b,
                      int32_t* flag, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_flag_cand, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, ccol,
                       base, count, j0, b, flag);
    SIC_CHECK_LAUNCH();
}

void launch_a2_k(const DevCSR& A, int64_t j0, int b, const double* WNC, int64_t nC,
                 const int32_t* cmap, double* K, int32_t* err, hipStream_t s) {
    hipLaunchKernelGGL(k_a2_k, dim3(b), dim3(256), 0, s, A.rowptr.p, A.col.p, A.val.p, j0, b, WNC,
                       nC, cmap, K, err);
    SIC_CHECK_LAUNCH();
}

void launch_dense_aii(const DevCSR& A, int64_t j0, int b, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_dense_aii, dim3(b), dim3(256), 0, s, A.rowptr.p, A.col.p, A.val.p, j0, b, out);
    SIC_CHECK_LAUNCH();
}

void launch_screen_coarse(int pass, const int64_t* crow, const int32_t* ccol, int64_t base,
                          int64_t j0, int b, double lam, const double* S_cand, const double* WII,
                          const double* WNC, int64_t nC, const int32_t* cmap, const double* AJ,
                          int32_t* ccount, const int64_t* colptr, int32_t* e_row, double* e_g,
                          double* e_s, double* e_a, double* e_w, int32_t* nflag, hipStream_t s) {
    hipLaunchKernelGGL(k_screen_coarse, dim3(b), dim3(64), 0, s, pass, crow, ccol, base, j0, b, lam,
                       S_cand, WII, WNC, nC, cmap, AJ, ccount, colptr, e_row, e_g, e_s, e_a, e_w,
                       nflag);
    SIC_CHECK_LAUNCH();
}

}  // namespace sic
