// Small dense float64 linear algebra for the line search (Section 6.1.2,
// eq. (logdet_blocks), App. A.1) and for the neighbour identity of App. A.2.
//
// Line search in whitened form.  With W_II = R R^T (R lower), B0 = W_II^{-1}
// and C(alpha) = B0 + alpha B1 + alpha^2 B2 (the Schur complement of
// A + alpha Delta on the block, eq. (logdet_blocks)):
//     R^T C(alpha) R = I + alpha E1 + alpha^2 E2,
//     E1 = R^T Delta_II R + K1 + K1^T,    K1 = R^T M R^{-T},  M = Delta_IN W_NI
//     E2 = K1 K1^T - R^T (Delta_IN W_NN Delta_NI) R
// so  log det(A + alpha Delta) - log det A = log det(I + alpha E1 + alpha^2 E2)
// and A + alpha Delta > 0 iff that matrix is PD (eq. (Schurs_PDness)).  The
// Cholesky of I + E keeps the identity implicit and sums log1p of the pivots,
// so the change keeps full relative accuracy however small the step.
#include "profiler.h"

namespace sic {

namespace {

constexpr int CH_NB = 256;        // largest block handled by the Cholesky kernel

// Cholesky tiling (the kernel, k_chol, is described where it is defined).
typedef double chol_d4 __attribute__((ext_vector_type(4)));

constexpr int CB = 16;                  // block size of the factorization
constexpr int CB_N = CH_NB / CB;        // block rows of the largest matrix
constexpr int CH_THREADS = 512;
constexpr int CH_WAVES = CH_THREADS / 64;
constexpr int CB_PLD = CB + 1;          // padded LDS row (17 doubles)

constexpr int CB_RLD = CB + 2;          // padded row of a staged L block (18 doubles)

struct CholShared {
    double Rk[CB_N][CB * CB_RLD];       // row block kb of L (the blocks left of the diagonal)
    double Pn[CB_N][CB * CB_PLD];       // updated blocks of column kb, accumulator layout
    double Part[CH_WAVES][4 * 64];      // partial sums when a block's K range is split
    double Lik[CB * CB_PLD];            // inverse of the diagonal factor (lower)
    double piv[CH_NB];                  // pivots (t of pivot 1 + t, or t), for the log det
    double red[CH_WAVES];
    int bad;
};

// Barrier for LDS traffic only: outstanding global stores and loads stay in
// flight across it.
__device__ inline void chol_lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// p[idx] when cond, else dflt, with the load itself unconditional (index 0
// when !cond, which must be a valid element): a predicated load would become
// a branch that waits for its data before the next load is issued.
__device__ inline double load_or(const double* __restrict__ p, int64_t idx, bool cond, double dflt) {
    const double v = p[cond ? idx : 0];
    return cond ? v : dflt;
}

__device__ inline double chol_readlane(double v, int l) {
    const long long bits = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(bits & 0xffffffffll), l);
    const int hi = __builtin_amdgcn_readlane((int)(bits >> 32), l);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// In-place lower Cholesky of one nb x nb matrix (nb <= 256) per workgroup
// (batch over blockIdx.x, matrices `stride` doubles apart, leading dimension
// ld), left-looking over 16-column block columns; the factor is written in
// place and re-read from there (the matrix stays in L2). For block column kb:
//   1. C_I = A_{I,kb} - sum_j L_{I,j} L_{kb,j}^T for every block row I >= kb
//      on FP64 MFMA (16x16x4), the L_{I,j} operands read from the stored
//      factor, all of a step's loads in flight at once; the waves of block
//      row kb also put their operands (row block kb of L) in LDS as the other
//      factor. When few block rows remain, their K ranges are split over the
//      waves and the partial sums added in a fixed order;
//   2. one wave factors C_kk (rows in lanes 0..15, the pivot row broadcast
//      with readlane) and inverts the factor (lane j forming column j, the
//      factor read back from LDS);
//   3. each panel block becomes L_I = C_I L_kk^{-T} (4 MFMAs) and is stored.
// Only the panel stores are re-read inside the kernel, so only the barrier
// that ends a block column waits for global stores.
// identity != 0 factors I + E: pivot = 1 + t, log det term = log1p(t).
// out[2*batch] = log det, out[2*batch+1] = 1 if PD else 0. Only the lower
// triangle is read; the factor overwrites it (partly, when not PD), the upper
// triangle of the diagonal blocks is zeroed and the blocks above them receive
// the transpose of the factor (the kernel's own operand copy; callers that
// need a clean lower factor zero them). dinv (batch 1 only, may be null): the
// inverses of the 16 x 16 diagonal blocks of the factor, block k at
// dinv + 256 k, row-major.
__global__ __launch_bounds__(CH_THREADS) void k_chol(double* __restrict__ M, int64_t stride,
                                                     int nb, int ld, int identity,
                                                     double* __restrict__ out,
                                                     double* __restrict__ dinv) {
    __shared__ CholShared sh;
    double* A = M + (int64_t)blockIdx.x * stride;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane >> 4, lc = lane & 15;
    const int nt = (nb + CB - 1) / CB;
    const double pad = identity ? 0.0 : 1.0;   // padded diagonal: contributes log 1 = 0
    if (tid == 0) sh.bad = 0;
    for (int kb = 0; kb < nt; ++kb) {
        const int r0 = kb * CB;
        // (1) C_I for I = kb .. nt-1. With nout >= 8 block rows, wave w takes rows
        // kb + w and kb + w + 8 (then kb <= 7); with fewer, ws waves split the K
        // range of one row (then at most 11 block columns per wave). Every load
        // of the step is issued before the staging barrier: the initial block
        // values and the L_{I,j} operands, 16 jobs of one block column each.
        const int nout = nt - kb;
        const int ws = nout >= CH_WAVES ? 1 : CH_WAVES / nout;
        const int groups = CH_WAVES / ws;
        const int slice = wave % ws;
        const int jlo = slice * kb / ws, jhi = (slice + 1) * kb / ws;
        const int I0 = kb + wave / ws, I1 = I0 + groups;
        const int nbw = I0 >= nt ? 0 : (ws == 1 && I1 < nt ? 2 : 1);
        chol_d4 acc0, acc1;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int col = r0 + lc;
            double v0 = 0.0, v1 = 0.0;
            const int row0 = I0 * CB + lr + 4 * v, row1 = I1 * CB + lr + 4 * v;
            const bool in0 = slice == 0 && nbw >= 1 && row0 < nb && col < nb && col <= row0;
            const bool in1 = slice == 0 && nbw == 2 && row1 < nb && col < nb;
            v0 = load_or(A, (int64_t)row0 * ld + col, in0, 0.0);
            v1 = load_or(A, (int64_t)row1 * ld + col, in1, 0.0);
            if (slice == 0 && nbw >= 1 && !(row0 < nb && col < nb) && row0 == col) v0 = pad;
            if (slice == 0 && nbw == 2 && !(row1 < nb && col < nb) && row1 == col) v1 = pad;
            acc0[v] = v0;
            acc1[v] = v1;
        }
        constexpr int JOBS = 16;
        double a[JOBS][4];
#pragma unroll
        for (int x = 0; x < JOBS; ++x) {
            const int q = nbw == 2 ? (x >> 3) : 0;
            const int j = jlo + (nbw == 2 ? (x & 7) : x);
            const bool valid = nbw >= 1 && j < jhi;
            // L_{I,j}[lc][4 lr + t], read from its transpose in the upper triangle so
            // that 16 consecutive lanes read one contiguous row segment
            // (valid is the same in every lane: jobs past the wave's range issue
            // nothing, which matters because the memory pipeline's cost is per
            // instruction). Lanes past nb read element 0 and are masked where
            // the values are used: a select here would wait for each load.
            const int acol = (q ? I1 : I0) * CB + lc;
            if (valid) {
#pragma unroll
                for (int t = 0; t < 4; ++t)
                    a[x][t] = A[acol < nb ? (int64_t)(j * CB + 4 * lr + t) * ld + acol : 0];
            } else {
#pragma unroll
                for (int t = 0; t < 4; ++t) a[x][t] = 0.0;
            }
        }
        // Rk[j][r][c] = -L[r0 + r][j*16 + c] (the B operands, row block kb of L,
        // negated so that the products subtract) from the waves whose block row
        // is kb: their A operands above are those blocks, read from the
        // transposed copy, so no load of its own is needed
        const bool in0c = I0 * CB + lc < nb, in1c = I1 * CB + lc < nb;   // lanes inside the matrix
        if (I0 == kb) {
#pragma unroll
            for (int x = 0; x < JOBS; ++x) {
                const int j = jlo + (nbw == 2 ? (x & 7) : x);
                if ((nbw == 1 || x < 8) && j < jhi) {
#pragma unroll
                    for (int t = 0; t < 4; ++t)
                        sh.Rk[j][lc * CB_RLD + 4 * lr + t] = in0c ? -a[x][t] : 0.0;
                }
            }
        }
        chol_lds_barrier();
#pragma unroll
        for (int x = 0; x < JOBS; ++x) {
            const int q = nbw == 2 ? (x >> 3) : 0;
            const int j = jlo + (nbw == 2 ? (x & 7) : x);
            if (nbw >= 1 && j < jhi) {
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const double bv = sh.Rk[j][lc * CB_RLD + 4 * lr + t];
                    const double av = (q ? in1c : in0c) ? a[x][t] : 0.0;
                    if (q)
                        acc1 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc1, 0, 0, 0);
                    else
                        acc0 = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc0, 0, 0, 0);
                }
            }
        }
        if (nbw >= 1) {
            if (ws > 1) {
#pragma unroll
                for (int v = 0; v < 4; ++v) sh.Part[wave][v * 64 + lane] = acc0[v];
            } else {
#pragma unroll
                for (int v = 0; v < 4; ++v) sh.Pn[I0][(lr + 4 * v) * CB_PLD + lc] = acc0[v];
            }
        }
        if (nbw == 2) {
#pragma unroll
            for (int v = 0; v < 4; ++v) sh.Pn[I1][(lr + 4 * v) * CB_PLD + lc] = acc1[v];
        }
        chol_lds_barrier();
        if (ws > 1 && slice == 0 && wave / ws < nout) {
            const int I = kb + wave / ws;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                double sacc = 0.0;
                for (int q = 0; q < ws; ++q) sacc += sh.Part[wave + q][v * 64 + lane];
                sh.Pn[I][(lr + 4 * v) * CB_PLD + lc] = sacc;
            }
        }
        chol_lds_barrier();
        // (3) factor and invert the diagonal block
        if (wave == 0) {
            const bool on = lane < CB;
            double rw[CB];
#pragma unroll
            for (int j = 0; j < CB; ++j) {
                const double v = sh.Pn[kb][(on ? lane : 0) * CB_PLD + j];
                rw[j] = on ? v : 0.0;
            }
            double tsave = 1.0;
            double ikks[CB];   // 1 / L_kk (uniform)
            int bad = 0;
#pragma unroll
            for (int k = 0; k < CB; ++k) {
                const double t = chol_readlane(rw[k], k);
                const double piv = identity ? 1.0 + t : t;
                if (!(piv > 0.0) || !isfinite(piv)) bad = 1;
                // 1/sqrt(piv): the hardware estimate and two Newton steps (each
                // doubles the correct bits), then sqrt(piv) = piv / sqrt(piv); a
                // third of the dependent operations of a rounded sqrt and divide
                double ikk = __builtin_amdgcn_rsq(piv);
                const double hp = 0.5 * piv;
#pragma unroll
                for (int it = 0; it < 2; ++it) ikk = fma(ikk, fma(-hp * ikk, ikk, 0.5), ikk);
                const double lkk = piv * ikk;
                ikks[k] = ikk;
                if (lane == k) tsave = t;
                rw[k] = (lane == k) ? lkk : rw[k] * ikk;   // lanes > k: L_ik
#pragma unroll
                for (int j = k + 1; j < CB; ++j) rw[j] -= rw[k] * chol_readlane(rw[k], j);
            }
            // The factor's rows go out, and to LDS transposed (T[k][i] = L_ik,
            // with 1/L_kk on the diagonal) in the partial-sum area, free now.
            // Then lane j forms column j of the inverse by forward substitution,
            // right-looking (once x_k is known every later row's sum takes
            // L_ik x_k, one broadcast read of T), each entry stored when formed.
            double* T = &sh.Part[0][0];
            if (on) {
                const int row = r0 + lane;
#pragma unroll
                for (int k = 0; k < CB; ++k) {
                    T[k * CB_PLD + lane] = (k == lane) ? ikks[k] : ((k < lane) ? rw[k] : 0.0);
                    if (row < nb && r0 + k < nb) A[(int64_t)row * ld + r0 + k] = (k <= lane) ? rw[k] : 0.0;
                }
            }
            // Row k + 1 of T is read at the start of step k, before the step's
            // stores, so its latency hides behind the step; the compiler
            // barrier keeps the reads from being hoisted further (all of T at
            // once would not fit the registers).
            double rs[CB], tn[CB];
#pragma unroll
            for (int i = 0; i < CB; ++i) {
                rs[i] = 0.0;
                tn[i] = T[i];
            }
#pragma unroll
            for (int k = 0; k < CB; ++k) {
                double tc[CB];
#pragma unroll
                for (int i = k; i < CB; ++i) tc[i] = tn[i];
                if (k + 1 < CB) {
#pragma unroll
                    for (int i = k + 1; i < CB; ++i) tn[i] = T[(k + 1) * CB_PLD + i];
                }
                const double x = ((lane == k ? 1.0 : 0.0) - rs[k]) * tc[k];
                if (on) {
                    const double iv = (k >= lane) ? x : 0.0;
                    sh.Lik[k * CB_PLD + lane] = iv;
                    if (dinv && !bad) dinv[kb * CB * CB + k * CB + lane] = iv;
                }
#pragma unroll
                for (int i = k + 1; i < CB; ++i) rs[i] = fma(tc[i], x, rs[i]);
                asm volatile("" ::: "memory");
            }
            if (on) sh.piv[kb * CB + lane] = tsave;
            if (lane == 0 && bad) sh.bad = 1;
        }
        chol_lds_barrier();   // the factor's global copy is not re-read in this kernel
        if (sh.bad) break;
        // (4) panel blocks L_I = C_I L_kk^{-T}
        for (int I = kb + 1 + wave; I < nt; I += CH_WAVES) {
            chol_d4 r = {0.0, 0.0, 0.0, 0.0};
            double a[4], bv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                a[t] = sh.Pn[I][lc * CB_PLD + 4 * lr + t];
                bv[t] = sh.Lik[lc * CB_PLD + 4 * lr + t];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) r = __builtin_amdgcn_mfma_f64_16x16x4f64(a[t], bv[t], r, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = I * CB + lr + 4 * v, col = r0 + lc;
                if (row < nb && col < nb) {
                    A[(int64_t)row * ld + col] = r[v];
                    A[(int64_t)col * ld + row] = r[v];   // transposed copy for later steps
                }
            }
        }
        __syncthreads();   // the new block column of L is visible to the next step
    }
    // log det: the log (log1p for I + E) of every pivot at once, summed in a
    // fixed order (the padded pivots contribute log 1 = 0)
    double lg = 0.0;
    if (!sh.bad && tid < nt * CB) lg = identity ? log1p(sh.piv[tid]) : log(sh.piv[tid]);
    for (int off = 32; off > 0; off >>= 1) lg += __shfl_xor(lg, off, 64);
    if (lane == 0) sh.red[wave] = lg;
    __syncthreads();
    if (tid == 0) {
        double ld_sum = 0.0;
        for (int w = 0; w < CH_WAVES; ++w) ld_sum += sh.red[w];
        out[2 * blockIdx.x] = sh.bad ? 0.0 : ld_sum;
        out[2 * blockIdx.x + 1] = sh.bad ? 0.0 : 1.0;
    }
}

// Solve L X = B (trans = 0) or L^T X = B (trans = 1) in place, with L the
// nb x nb lower Cholesky factor written by k_chol (leading dimension ldl) and
// dinv the inverses of its 16 x 16 diagonal blocks; B is nb x ncols row-major
// (leading dimension ldb). Blocked substitution over 16-row blocks: block i
// of X is dinv_i (B_i - sum_{j<i} L_ij X_j) (forward) or
// dinv_i^T (B_i - sum_{j>i} L_ji^T X_j) (backward). One workgroup solves
// TS_COLS right-hand sides, held in LDS. The sum over j is a product on FP64
// MFMA (16x16x4), its 16-column K blocks split over the four waves and the
// partial sums added in a fixed order; wave 0 then applies dinv_i, also on
// MFMA.
constexpr int TS_COLS = 16;
constexpr int TS_T = CB;   // the factor's diagonal-block size (dinv layout)
constexpr int TS_THREADS = TS_COLS * TS_T;
static_assert(TS_THREADS == TS_T * TS_T, "one diagonal-block entry per thread");
static_assert(TS_THREADS == 4 * 64, "the partial sums are added as four waves");

__global__ __launch_bounds__(TS_THREADS) void k_trsm_blocked(const double* __restrict__ L, int nb,
                                                             int ldl, const double* __restrict__ dinv,
                                                             double* __restrict__ B, int ncols,
                                                             int ldb, int trans) {
    constexpr int LPT = (TS_T * CH_NB + TS_THREADS - 1) / TS_THREADS;   // staged L per thread
    __shared__ double Xs[CH_NB][TS_COLS];
    __shared__ double Ls[TS_T * CH_NB];   // the L entries of the current step (see below)
    __shared__ double As[TS_T][TS_COLS];
    __shared__ double Ds[TS_T * TS_T];    // inverse of the step's diagonal block
    __shared__ double Part[TS_THREADS / 64][TS_T * TS_COLS];   // the waves' partial sums
    const int tid = threadIdx.x;
    const int r = tid / TS_COLS, c = tid % TS_COLS;
    const int col = blockIdx.x * TS_COLS + c;
    const bool con = col < ncols;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lr = lane >> 4, lc = lane & 15;   // MFMA operand lanes (as in k_chol)
    const int nt = (nb + TS_T - 1) / TS_T;
    for (int k = r; k < nt * TS_T; k += TS_T)
        Xs[k][c] = load_or(B, (int64_t)k * ldb + col, con && k < nb, 0.0);
    // the L entries a step needs, with every load in flight at once:
    //   forward:  Ls[q * 16 + rr] = L[i*16 + rr][q]           for q <  i*16
    //   backward: Ls[q * 16 + rr] = L[(i+1)*16 + q][i*16 + rr] for q <  nb - (i+1)*16
    // They do not depend on X: step + 1's are loaded into registers while step
    // runs, so no step waits for global memory but the first.
    double lreg[LPT];
    double dv = 0.0;
    auto load_step = [&](int i) {
        const int kcnt = trans ? nb - (i + 1) * TS_T : i * TS_T;
#pragma unroll
        for (int u = 0; u < LPT; ++u) {
            const int e = tid + TS_THREADS * u;
            const int q = e / TS_T, rr = e % TS_T;
            const int row = trans ? (i + 1) * TS_T + q : i * TS_T + rr;
            const int lc = trans ? i * TS_T + rr : q;
            const bool ok = q < kcnt && row < nb && lc < nb;
            lreg[u] = load_or(L, (int64_t)row * ldl + lc, ok, 0.0);
        }
        dv = dinv[(int64_t)i * TS_T * TS_T + tid];   // TS_THREADS == TS_T * TS_T
    };
    load_step(trans ? nt - 1 : 0);
    for (int step = 0; step < nt; ++step) {
        const int i = trans ? nt - 1 - step : step;
        const int kcnt = trans ? nb - (i + 1) * TS_T : i * TS_T;
#pragma unroll
        for (int u = 0; u < LPT; ++u) {
            const int e = tid + TS_THREADS * u;
            if (e < TS_T * CH_NB) Ls[e] = lreg[u];
        }
        Ds[tid] = dv;
        __syncthreads();
        if (step + 1 < nt) load_step(trans ? nt - 2 - step : step + 1);
        const int k0 = trans ? (i + 1) * TS_T : 0;
        // partial sum of L_i. X over the K blocks jb = wave, wave + 4, ...: the
        // A operand is Ls[q][m] (zero past kcnt), the B operand X[k0 + q][n]
        const int nkb = (kcnt + TS_T - 1) / TS_T;
        chol_d4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int jb = wave; jb < nkb; jb += TS_THREADS / 64) {
            double av[4], bv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int q = jb * TS_T + 4 * lr + t;
                av[t] = Ls[q * TS_T + lc];
                bv[t] = Xs[k0 + q][lc];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t], bv[t], acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; ++v) Part[wave][(lr + 4 * v) * TS_COLS + lc] = acc[v];
        __syncthreads();
        if (wave == 0) {
            // A_i = B_i - the partial sums (rows lr + 4 v, column lc), then
            // X_i = dinv_i A_i (dinv_i^T A_i backward) through As
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rr = lr + 4 * v, row = i * TS_T + rr;
                const int o = rr * TS_COLS + lc;
                const double s4 = (Part[0][o] + Part[1][o]) + (Part[2][o] + Part[3][o]);
                As[rr][lc] = row < nb ? Xs[row][lc] - s4 : 0.0;
            }
            chol_d4 x = {0.0, 0.0, 0.0, 0.0};
            double dv[4], bv[4];
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int q = 4 * lr + t;
                dv[t] = trans ? Ds[q * TS_T + lc] : Ds[lc * TS_T + q];
                bv[t] = As[q][lc];
            }
#pragma unroll
            for (int t = 0; t < 4; ++t) x = __builtin_amdgcn_mfma_f64_16x16x4f64(dv[t], bv[t], x, 0, 0, 0);
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int row = i * TS_T + lr + 4 * v;
                if (row < nb) Xs[row][lc] = x[v];
            }
        }
        __syncthreads();
    }
    if (con)
        for (int k = r; k < nb; k += TS_T) B[(int64_t)k * ldb + col] = Xs[k][c];
}

// C = alpha * op(A) op(B) + beta * C on FP64 MFMA (16x16x4): one workgroup of
// four waves per 32 x 32 tile of C (each wave one 16 x 16 accumulator), K
// staged through LDS 16 at a time with the next stage's loads in flight
// during the current stage's products. op(X) = X or X^T; row-major with
// leading dimensions.
typedef double gemm_d4 __attribute__((ext_vector_type(4)));
constexpr int GM_TILE = 32, GM_KC = 16, GM_PAD = 4;

__global__ __launch_bounds__(256) void k_gemm_mfma(int M, int N, int K, double alpha,
                                                   const double* __restrict__ A, int lda, int ta,
                                                   const double* __restrict__ B, int ldb, int tb,
                                                   double beta, double* __restrict__ C, int ldc) {
    __shared__ double sA[GM_KC][GM_TILE + GM_PAD];   // sA[k][i] = op(A)[i0 + i][k0 + k]
    __shared__ double sB[GM_KC][GM_TILE + GM_PAD];   // sB[k][j] = op(B)[k0 + k][j0 + j]
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int i0 = blockIdx.y * GM_TILE, j0 = blockIdx.x * GM_TILE;
    const int lr = tid >> 4;          // 0..15 (k within the stage)
    const int lc = (tid & 15) * 2;    // 0..30 (i or j within the tile)
    gemm_d4 acc = {0.0, 0.0, 0.0, 0.0};
    double va[2], vb[2];
    auto load_stage = [&](int k0) {
        const int k = k0 + lr;
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int i = i0 + lc + q, j = j0 + lc + q;
            const int64_t ia = ta ? (int64_t)k * lda + i : (int64_t)i * lda + k;
            const int64_t ib = tb ? (int64_t)j * ldb + k : (int64_t)k * ldb + j;
            va[q] = load_or(A, ia, i < M && k < K, 0.0);
            vb[q] = load_or(B, ib, j < N && k < K, 0.0);
        }
    };
    load_stage(0);
    for (int k0 = 0; k0 < K; k0 += GM_KC) {
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            sA[lr][lc + q] = va[q];
            sB[lr][lc + q] = vb[q];
        }
        __syncthreads();
        load_stage(k0 + GM_KC);   // beyond K: guarded loads of element 0
#pragma unroll
        for (int kk = 0; kk < GM_KC; kk += 4) {
            const int kr = kk + (lane >> 4);
            const double av = sA[kr][wr * 16 + (lane & 15)];
            const double bv = sB[kr][wc * 16 + (lane & 15)];
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
        __syncthreads();
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
        const int i = i0 + wr * 16 + (lane >> 4) + 4 * v;
        const int j = j0 + wc * 16 + (lane & 15);
        if (i < M && j < N) {
            const int64_t o = (int64_t)i * ldc + j;
            const double prev = beta != 0.0 ? C[o] : 0.0;
            C[o] = alpha * acc[v] + beta * prev;
        }
    }
}


// Copy the leading nb x nb block of a (ld) matrix into a packed nb x nb buffer.
__global__ void k_copy_block(const double* __restrict__ src, int ld, int nb, double* __restrict__ dst) {
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < nb; j += blockDim.x) dst[(int64_t)i * nb + j] = src[(int64_t)i * ld + j];
}

// Delta_II as a dense symmetric b x b matrix from the coordinates with p < b.
__global__ void k_ls_d11(const int64_t* __restrict__ cptr, const int32_t* __restrict__ c_p,
                         const double* __restrict__ delta, int b, double* __restrict__ D11) {
    const int ci = blockIdx.x;
    for (int64_t t = cptr[ci] + threadIdx.x; t < cptr[ci + 1]; t += blockDim.x) {
        const int p = c_p[t];
        if (p < b) {
            D11[(int64_t)p * b + ci] = delta[t];
            D11[(int64_t)ci * b + p] = delta[t];
        }
    }
}

// M[c][q] = sum_{t in column c, p_t in N} Delta_t W[p_t][q],  q < b   (M = Delta_IN W_NI)
__global__ void k_ls_m(const int64_t* __restrict__ cptr, const int32_t* __restrict__ c_p,
                       const double* __restrict__ delta, const double* __restrict__ WJJ, int jp,
                       int b, double* __restrict__ Mo) {
    const int ci = blockIdx.x;
    for (int q = threadIdx.x; q < b; q += blockDim.x) {
        double s = 0.0;
        for (int64_t t = cptr[ci]; t < cptr[ci + 1]; ++t) {
            const int p = c_p[t];
            if (p >= b) s += delta[t] * WJJ[(int64_t)p * jp + q];
        }
        Mo[(int64_t)ci * b + q] = s;
    }
}

// Y[pp][c] = sum_{t in column c, p_t in N} W[b+pp][p_t] Delta_t   (Y = W_NN Delta_NI, nN x b)
__global__ void k_ls_y(const int64_t* __restrict__ cptr, const int32_t* __restrict__ c_p,
                       const double* __restrict__ delta, const double* __restrict__ WJJ, int jp,
                       int b, int nN, double* __restrict__ Y) {
    const int ci = blockIdx.y;
    const int pp = blockIdx.x * blockDim.x + threadIdx.x;
    if (pp >= nN) return;
    const double* wrow = WJJ + (int64_t)(b + pp) * jp;
    double s = 0.0;
    for (int64_t t = cptr[ci]; t < cptr[ci + 1]; ++t) {
        const int p = c_p[t];
        if (p >= b) s += wrow[p] * delta[t];
    }
    Y[(int64_t)pp * b + ci] = s;
}

// P[c][c'] = sum_{t in column c, p_t in N} Delta_t Y[p_t - b][c']   (P = Delta_IN W_NN Delta_NI)
__global__ void k_ls_p(const int64_t* __restrict__ cptr, const int32_t* __restrict__ c_p,
                       const double* __restrict__ delta, const double* __restrict__ Y, int b,
                       double* __restrict__ P) {
    const int ci = blockIdx.x;
    for (int q = threadIdx.x; q < b; q += blockDim.x) {
        double s = 0.0;
        for (int64_t t = cptr[ci]; t < cptr[ci + 1]; ++t) {
            const int p = c_p[t];
            if (p >= b) s += delta[t] * Y[(int64_t)(p - b) * b + q];
        }
        P[(int64_t)ci * b + q] = s;
    }
}

// E1 = D1 + X + X^T (X = K1^T), E2 = XtX - RPR, both symmetrised.
__global__ void k_ls_e(const double* __restrict__ D1, const double* __restrict__ X,
                       const double* __restrict__ XtX, const double* __restrict__ RPR, int b,
                       double* __restrict__ E1, double* __restrict__ E2) {
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < b; j += blockDim.x) {
        const int64_t o = (int64_t)i * b + j, ot = (int64_t)j * b + i;
        E1[o] = 0.5 * (D1[o] + D1[ot]) + X[o] + X[ot];
        E2[o] = 0.5 * (XtX[o] + XtX[ot]) - 0.5 * (RPR[o] + RPR[ot]);
    }
}

// Trial steps are alpha = 2^-(first + trial), formed exactly on the device.
__global__ void k_ls_trials(const double* __restrict__ E1, const double* __restrict__ E2, int b,
                            int first, double* __restrict__ C) {
    const int trial = blockIdx.y;
    const int i = blockIdx.x;
    const double a = ldexp(1.0, -(first + trial));
    double* Ct = C + (int64_t)trial * b * b;
    for (int j = threadIdx.x; j < b; j += blockDim.x) {
        const int64_t o = (int64_t)i * b + j;
        Ct[o] = a * E1[o] + a * a * E2[o];
    }
}

__device__ inline double abs_change(double a, double d) {
    // |a + d| - |a| without rounding a + d when the sign is kept
    if (a != 0.0) {
        const double s = a + d;
        if ((s > 0.0) == (a > 0.0) && s != 0.0) return a > 0.0 ? d : -d;
        return fabs(s) - fabs(a);
    }
    return fabs(d);
}

// lin[trial] = sum_t w_t (alpha S_t Delta_t + lam (|A_t + alpha Delta_t| - |A_t|)),
// w_t = 1 on the diagonal, 2 off it (both triangles of the pair).
__global__ __launch_bounds__(256) void k_ls_linear(int64_t ncoord, const int32_t* __restrict__ c_p,
                                                   const int32_t* __restrict__ c_ci,
                                                   const double* __restrict__ c_S,
                                                   const double* __restrict__ c_A,
                                                   const double* __restrict__ delta, double lam,
                                                   int first, double* __restrict__ lin) {
    __shared__ double red[256];
    const double a = ldexp(1.0, -(first + (int)blockIdx.x));
    double s = 0.0;
    for (int64_t t = threadIdx.x; t < ncoord; t += 256) {
        const double w = (c_p[t] == c_ci[t]) ? 1.0 : 2.0;
        const double d = delta[t];
        s += w * (a * c_S[t] * d + lam * abs_change(c_A[t], a * d));
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) lin[blockIdx.x] = red[0];
}

__global__ void k_zero_upper(double* __restrict__ M, int nb, int ld) {
    const int i = blockIdx.x;
    for (int j = i + 1 + threadIdx.x; j < nb; j += blockDim.x) M[(int64_t)i * ld + j] = 0.0;
}

__global__ void k_identity_minus(const double* __restrict__ K, int b, double* __restrict__ out) {
    const int i = blockIdx.x;
    for (int j = threadIdx.x; j < b; j += blockDim.x)
        out[(int64_t)i * b + j] = (i == j ? 1.0 : 0.0) - K[(int64_t)i * b + j];
}

}  // namespace

// Scatter a full symmetric CSR into a dense n x n row-major matrix (zeroed
// first): one workgroup per row.
__global__ void k_csr_to_dense(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                               const double* __restrict__ val, int64_t n, double* __restrict__ D) {
    const int64_t i = blockIdx.x;
    double* row = D + i * n;
    for (int64_t j = threadIdx.x; j < n; j += blockDim.x) row[j] = 0.0;
    __syncthreads();
    for (int64_t e = rowptr[i] + threadIdx.x; e < rowptr[i + 1]; e += blockDim.x) row[col[e]] = val[e];
}

void launch_csr_to_dense(const int64_t* rowptr, const int32_t* col, const double* val, int64_t n,
                         double* D, hipStream_t s) {
    hipLaunchKernelGGL(k_csr_to_dense, dim3((unsigned)n), dim3(256), 0, s, rowptr, col, val, n, D);
    SIC_CHECK_LAUNCH();
}

void launch_zero_upper(double* M, int nb, int ld, hipStream_t s) {
    if (nb <= 1) return;
    hipLaunchKernelGGL(k_zero_upper, dim3(nb), dim3(256), 0, s, M, nb, ld);
    SIC_CHECK_LAUNCH();
}

void launch_identity_minus(const double* K, int b, double* out, hipStream_t s) {
    hipLaunchKernelGGL(k_identity_minus, dim3(b), dim3(256), 0, s, K, b, out);
    SIC_CHECK_LAUNCH();
}

void launch_chol(double* M, int64_t stride, int batch, int nb, int ld, int identity, double* out,
                 hipStream_t s, double* dinv) {
    if (nb > CH_NB) throw SicError(SIC_ETOOBIG, "block larger than the Cholesky kernel supports");
    if (dinv && batch != 1) throw SicError(SIC_EINTERNAL, "diagonal-tile inverses need batch 1");
    prof_begin(KK_CHOL, s);
    hipLaunchKernelGGL(k_chol, dim3(batch), dim3(CH_THREADS), 0, s, M, stride, nb, ld, identity, out,
                       dinv);
    SIC_CHECK_LAUNCH();
    prof_end(KK_CHOL, s, 16.0 * nb * nb * (double)batch, (double)nb * nb * nb / 3.0 * batch);
}

void launch_trsm_lower(const double* L, int nb, int ldl, const double* dinv, double* B, int ncols,
                       int ldb, int trans, hipStream_t s) {
    if (ncols <= 0 || nb <= 0) return;
    if (nb > CH_NB) throw SicError(SIC_ETOOBIG, "block larger than the triangular solve supports");
    prof_begin(KK_TRSM, s);
    hipLaunchKernelGGL(k_trsm_blocked, dim3((unsigned)((ncols + TS_COLS - 1) / TS_COLS)),
                       dim3(TS_THREADS), 0, s, L, nb, ldl, dinv, B, ncols, ldb, trans);
    SIC_CHECK_LAUNCH();
    // the triangle of L once per workgroup (from L2), B read and written once
    prof_end(KK_TRSM, s, 8.0 * (double)nb * nb / 2.0 + 16.0 * (double)nb * ncols,
             (double)nb * nb * ncols);
}

void launch_gemm_small(int M, int N, int K, double alpha, const double* A, int lda, int ta,
                       const double* B, int ldb, int tb, double beta, double* C, int ldc,
                       hipStream_t s) {
    if (M <= 0 || N <= 0) return;
    dim3 grid((unsigned)((N + GM_TILE - 1) / GM_TILE), (unsigned)((M + GM_TILE - 1) / GM_TILE));
    prof_begin(KK_GEMM, s);
    hipLaunchKernelGGL(k_gemm_mfma, grid, dim3(256), 0, s, M, N, K, alpha, A, lda, ta, B, ldb, tb,
                       beta, C, ldc);
    SIC_CHECK_LAUNCH();
    prof_end(KK_GEMM, s, 8.0 * ((double)M * K + (double)K * N + 2.0 * M * N), 2.0 * (double)M * N * K);
}

void launch_copy_block(const double* src, int ld, int nb, double* dst, hipStream_t s) {
    if (nb <= 0) return;
    hipLaunchKernelGGL(k_copy_block, dim3(nb), dim3(256), 0, s, src, ld, nb, dst);
    SIC_CHECK_LAUNCH();
}

void launch_ls_terms(const int64_t* cptr, const int32_t* c_p, const double* delta,
                     const double* WJJ, int jp, int b, int nN, double* D11, double* Mo, double* Y,
                     double* P, hipStream_t s) {
    SIC_HIP(hipMemsetAsync(D11, 0, sizeof(double) * b * b, s));
    hipLaunchKernelGGL(k_ls_d11, dim3(b), dim3(64), 0, s, cptr, c_p, delta, b, D11);
    SIC_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_ls_m, dim3(b), dim3(256), 0, s, cptr, c_p, delta, WJJ, jp, b, Mo);
    SIC_CHECK_LAUNCH();
    if (nN > 0) {
        hipLaunchKernelGGL(k_ls_y, dim3((unsigned)((nN + 255) / 256), (unsigned)b), dim3(256), 0, s,
                           cptr, c_p, delta, WJJ, jp, b, nN, Y);
        SIC_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_ls_p, dim3(b), dim3(256), 0, s, cptr, c_p, delta, Y, b, P);
        SIC_CHECK_LAUNCH();
    } else {
        SIC_HIP(hipMemsetAsync(P, 0, sizeof(double) * b * b, s));
    }
}

void launch_ls_e(const double* D1, const double* X, const double* XtX, const double* RPR, int b,
                 double* E1, double* E2, hipStream_t s) {
    hipLaunchKernelGGL(k_ls_e, dim3(b), dim3(256), 0, s, D1, X, XtX, RPR, b, E1, E2);
    SIC_CHECK_LAUNCH();
}

void launch_ls_trials(const double* E1, const double* E2, int b, int first, int ntrial,
                      double* C, hipStream_t s) {
    hipLaunchKernelGGL(k_ls_trials, dim3(b, ntrial), dim3(256), 0, s, E1, E2, b, first, C);
    SIC_CHECK_LAUNCH();
}

void launch_ls_linear(int64_t ncoord, const int32_t* c_p, const int32_t* c_ci, const double* c_S,
                      const double* c_A, const double* delta, double lam, int first,
                      int ntrial, double* lin, hipStream_t s) {
    hipLaunchKernelGGL(k_ls_linear, dim3(ntrial), dim3(256), 0, s, ncoord, c_p, c_ci, c_S, c_A, delta,
                       lam, first, lin);
    SIC_CHECK_LAUNCH();
}

}  // namespace sic
