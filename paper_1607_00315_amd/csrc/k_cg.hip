// Inverse columns W_J = A^{-1} E_J by conjugate gradients (Section 6.1, where
// these solves are the main cost of a block update and CG, possibly
// preconditioned, is the method named). Jacobi preconditioner (diag A > 0 for
// SPD A). A direction with p.Ap <= 0 while r != 0 (CG breakdown) proves A is
// not positive definite; the tile is then marked bad and stops.
//
// All k right-hand sides run together on row-major n x k blocks, so that one
// sparse row of A gathers whole 64-column segments of the direction block
// (coalesced 512-byte reads) and the per-column CG scalars stay independent.
// One iteration is two launches; each finishes the previous launch's
// per-column sums in its prologue (every workgroup of a column tile sums the
// same partials in the same order, so all take the same decision):
//   spmm(it):   rz, rr of the last update -> convergence of the tile (it > 0),
//               beta = rz / rz_old; p = z + beta p, q = A z + beta q (= A p),
//               partial p.q
//   update(it): alpha = rz / p.q; x += alpha p, r -= alpha q,
//               partial r.z, r.r (z = D^{-1} r is formed where it is read)
// rz alternates between two slots by iteration parity, so no launch reads a
// scalar that the same launch writes. No device-scope fences (they would
// write back the L2 of each XCD), no atomics: results do not depend on
// scheduling. Convergence is tracked per 64-column tile; launches for a
// converged tile return at once.
#include <mutex>

#include "profiler.h"

namespace sic {

namespace {

constexpr int CG_THREADS = 512;     // 8 waves, one matrix row per wave at a time
constexpr int CG_WAVES = CG_THREADS / 64;
constexpr int CG_ROW_TILES = 128;   // row partitions (partials per column)
constexpr int CG_TPW = CG_ROW_TILES / CG_WAVES;   // partials each wave sums per column
// gathers per row issued before their products: 8, or 16 for matrices whose
// rows average more than CG_WIDE_ROW entries (dense-regime iterates)
constexpr int CG_WIDE_ROW = 12;
constexpr int CG_UROWS = 4;         // rows per wave in flight in the update
constexpr int CG_SROWS = 1;         // rows per wave in flight in the product

// per-tile control block: [0] done, [1] iterations finished, [2] breakdown
// (p.Ap <= 0 with r.z > 0 in some column: A is not positive definite)
enum { T_DONE = 0, T_ITER = 1, T_BAD = 2, T_INTS = 3 };
enum { S_RZ0 = 0, S_RZ1 = 1, S_RR = 3 };   // rz by iteration parity; r.r

__global__ void k_cg_dinv(const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
                          const double* __restrict__ val, int64_t n, double* __restrict__ dinv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = 0.0;
    for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
        if (col[e] == (int32_t)i) d = val[e];
    dinv[i] = d > 0.0 ? 1.0 / d : 1.0;
}

// The product's coefficients with the preconditioner folded in:
// vd[e] = a_ic d_c, so that (A z)_i = sum_e vd[e] r_c with z = D^{-1} r.
__global__ void k_cg_vd(const int32_t* __restrict__ col, const double* __restrict__ val,
                        const double* __restrict__ dinv, int64_t nnz, double* __restrict__ vd) {
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x)
        vd[e] = val[e] * dinv[col[e]];
}

template <typename V>
__global__ void k_cg_init(int64_t n, int k, int col_tiles, const int32_t* __restrict__ cols,
                          const double* __restrict__ dinv, double* __restrict__ W,
                          V* __restrict__ R, double* __restrict__ scal,
                          int* __restrict__ tctl, double* __restrict__ tres,
                          int* __restrict__ mctl, double* __restrict__ mres, int fill) {
    // x0 = 0, r0 = e_cols[j] over the whole n x k block (rows over workgroups,
    // columns over threads), unless a warm start writes both (fill = 0);
    // z0 = D^{-1} r0 is formed where it is read
    for (int64_t i = blockIdx.x; fill && i < n; i += gridDim.x) {
        for (int j = threadIdx.x; j < k; j += blockDim.x) {
            const int64_t o = i * k + j;
            W[o] = 0.0;
            R[o] = cols[j] == i ? (V)1.0 : (V)0.0;
        }
    }
    if (blockIdx.x == 0) {
        for (int j = threadIdx.x; j < k; j += blockDim.x) {
            const int64_t c = cols[j];
            scal[j * 4 + S_RZ0] = (c >= 0 && c < n) ? dinv[c] : 0.0;
            scal[j * 4 + S_RZ1] = 0.0;
            scal[j * 4 + 2] = 0.0;
            scal[j * 4 + S_RR] = 1.0;
        }
        for (int j = threadIdx.x; j < col_tiles; j += blockDim.x) {
            tctl[j * T_INTS + T_DONE] = 0;
            tctl[j * T_INTS + T_ITER] = 0;
            tctl[j * T_INTS + T_BAD] = 0;
            tres[j] = 1.0;
            if (mctl) {
                mctl[j * T_INTS + T_DONE] = 0;
                mctl[j * T_INTS + T_ITER] = 0;
                mctl[j * T_INTS + T_BAD] = 0;
                mres[j] = 1.0;
            }
        }
    }
}

__device__ inline int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); }

// Warm start from the store of inverse columns: x0[:, j] = Ws[cols[j], :]
// (row c of the store holds column c of A^{-1}, which is symmetric) when the
// store holds column cols[j], else 0 (p and q start from zero in the first
// product after it). One 64 x 64 tile per workgroup, transposed through LDS so
// both sides are read and written in contiguous runs.
__global__ __launch_bounds__(256) void k_cg_warm(int64_t n, int k, const int32_t* __restrict__ cols,
                                                 const double* __restrict__ Ws,
                                                 const unsigned char* __restrict__ valid,
                                                 double* __restrict__ W) {
    __shared__ double t[64][65];
    const int64_t i0 = (int64_t)blockIdx.y * 64;
    const int j0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;   // 64 x 4 threads
    for (int jr = ty; jr < 64; jr += 4) {
        const int j = j0 + jr;
        const int64_t c = j < k ? cols[j] : -1;
        const bool ok = c >= 0 && c < n && valid[c] && i0 + tx < n;
        t[jr][tx] = ok ? Ws[c * n + i0 + tx] : 0.0;
    }
    __syncthreads();
    for (int ir = ty; ir < 64; ir += 4) {
        const int64_t i = i0 + ir;
        const int j = j0 + tx;
        if (i < n && j < k) W[i * k + j] = t[tx][ir];
    }
}

// The converged columns back into the store: Ws[cols[j], :] = x[:, j].
__global__ __launch_bounds__(256) void k_cg_store(int64_t n, int k, const int32_t* __restrict__ cols,
                                                  const double* __restrict__ W,
                                                  double* __restrict__ Ws,
                                                  unsigned char* __restrict__ valid) {
    __shared__ double t[64][65];
    const int64_t i0 = (int64_t)blockIdx.y * 64;
    const int j0 = blockIdx.x * 64;
    const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
    for (int ir = ty; ir < 64; ir += 4) {
        const int64_t i = i0 + ir;
        const int j = j0 + tx;
        t[ir][tx] = (i < n && j < k) ? W[i * k + j] : 0.0;
    }
    __syncthreads();
    for (int jr = ty; jr < 64; jr += 4) {
        const int j = j0 + jr;
        if (j >= k) continue;
        const int64_t c = cols[j];
        if (c < 0 || c >= n) continue;
        if (i0 + tx < n) Ws[c * n + i0 + tx] = t[tx][jr];
        if (blockIdx.y == 0 && tx == 0) valid[c] = 1;
    }
}


// The preconditioned residual z = D^{-1} r of one entry, rounded to the
// vector type (the value a stored z would hold). It is formed wherever it is
// read instead of being stored (one n x k array less written and read per
// iteration); the product's gathers take D^{-1} folded into the
// coefficients (k_cg_vd), so they read r alone.
template <typename V>
__device__ inline double zval(double di, V r) {
    return (double)(V)(di * (double)r);
}

// Tile of a workgroup (tx = 64-column tile, ty = row tile of `rows_per`
// contiguous rows). Workgroup L of a 1-D grid runs on XCD L % 8 (round-robin
// dispatch). mode 0: a plain gx x gy grid. mode 1 (column-grouped, gx >= 8):
// every row tile of one column tile on the same XCD, one column tile after
// another. mode 2 (row-banded, gy a multiple of 8): XCD x takes the gy / 8
// contiguous row tiles of band x, for every column tile. In both grouped
// modes the rows a tile gathers (its own and, on graphs with locality, their
// neighbours) come from one XCD's L2 instead of being fetched by several.
struct Tile {
    int tx, ty;
    bool ok;
};
__device__ inline Tile cg_tile(int mode, int gx, int gy) {
    Tile t;
    if (mode == 0) {
        t.tx = blockIdx.x;
        t.ty = blockIdx.y;
        t.ok = true;
        return t;
    }
    const int L = blockIdx.x, q = L & 7, slot = L >> 3;
    if (mode == 1) {
        const int c = slot / gy;
        t.ty = slot - c * gy;
        t.tx = q + 8 * c;
    } else {
        const int per = gy >> 3;
        const int c = slot / per;
        t.ty = q * per + (slot - c * per);
        t.tx = c;
    }
    t.ok = t.tx < gx;
    return t;
}

template <typename V, int CG_GATHER>
__global__ __launch_bounds__(CG_THREADS) void k_cg_spmm(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ vd, int64_t n, int k, const double* __restrict__ dinv,
    const V* __restrict__ R, V* __restrict__ P, V* __restrict__ Q, double* __restrict__ scal,
    const double* __restrict__ rzrr, double* __restrict__ part, int* __restrict__ tctl,
    double* __restrict__ tres, int* __restrict__ mctl, double* __restrict__ mres, double tol,
    int it, int restart, int gx, int gy, int64_t rows_per, int mode, int check_only) {
    const Tile T = cg_tile(mode, gx, gy);
    if (!T.ok) return;
    const int tx = T.tx, ty = T.ty;
    if (tctl[tx * T_INTS + T_DONE]) return;
    // first: no residual sums yet (a cold start's iteration 0); fresh: p and q
    // start from zero here (iteration 0, or the first after a warm start)
    const bool first = it == 0;
    const bool fresh = it == restart;
    const int lane = threadIdx.x & 63;
    const int wave = wave_id();
    const int j = tx * 64 + lane;
    const bool jok = j < k;
    const int jj = jok ? j : k - 1;   // clamped: every lane loads, masked lanes discard
    double beta = 0.0;
    if (!first) {
        // r.z and r.r of the last update (fixed order: row tiles t = w mod 8
        // in wave w, then the waves in order)
        // (all of a wave's partials are loaded before the first is added: a
        // rolled loop would wait for each load in turn)
        __shared__ double rsum[2][CG_WAVES][64];
        double v0[CG_TPW], v1[CG_TPW];
#pragma unroll
        for (int u = 0; u < CG_TPW; ++u) {
            const int t = wave + CG_WAVES * u;
            const int64_t o = ((int64_t)(t < gy ? t : 0) * k + jj) * 2;
            v0[u] = rzrr[o];
            v1[u] = rzrr[o + 1];
        }
        double a0 = 0.0, a1 = 0.0;
#pragma unroll
        for (int u = 0; u < CG_TPW; ++u) {
            if (wave + CG_WAVES * u < gy) {
                a0 += v0[u];
                a1 += v1[u];
            }
        }
        rsum[0][wave][lane] = a0;
        rsum[1][wave][lane] = a1;
        __syncthreads();
        double rz = 0.0, rr = 0.0;
        for (int w = 0; w < CG_WAVES; ++w) {
            rz += rsum[0][w][lane];
            rr += rsum[1][w][lane];
        }
        double res = jok ? sqrt(rr) : 0.0;
        for (int off = 32; off > 0; off >>= 1) res = fmax(res, __shfl_xor(res, off, 64));
        const double rz_old = scal[jj * 4 + ((it - 1) & 1)];
        beta = (jok && rz_old > 0.0) ? rz / rz_old : 0.0;
        const bool conv = res <= tol;   // the same in every workgroup of the tile
        if (ty == 0 && wave == 0) {     // the tile's record, for the host and update(it)
            if (jok) {
                scal[j * 4 + (it & 1)] = rz;
                scal[j * 4 + S_RR] = rr;
            }
            if (lane == 0) {
                const int itv = (conv || check_only) ? it : it + 1;
                tres[tx] = res;
                tctl[tx * T_INTS + T_ITER] = itv;
                if (conv) tctl[tx * T_INTS + T_DONE] = 1;
                if (mctl) {   // the host's copy (pinned memory), read at its next check
                    mres[tx] = res;
                    mctl[tx * T_INTS + T_ITER] = itv;
                    if (conv) mctl[tx * T_INTS + T_DONE] = 1;
                }
            }
        }
        if (conv) return;
    }
    if (check_only) return;
    double pq = 0.0;
    const int64_t r0 = (int64_t)ty * rows_per;
    const int64_t r1 = r0 + rows_per < n ? r0 + rows_per : n;
    // CG_SROWS rows per wave at a time (i, i + 8, ...), their gathers issued
    // together in batches of CG_GATHER per row. A short batch repeats the row's last entry with a zero
    // coefficient; a missing row repeats row i and is not stored.
    for (int64_t i = r0 + wave; i < r1; i += CG_SROWS * CG_WAVES) {
        bool has[CG_SROWS];
        int64_t e0[CG_SROWS], ne[CG_SROWS], o[CG_SROWS];
        double zo[CG_SROWS], po[CG_SROWS], qo[CG_SROWS], acc[CG_SROWS];
        int64_t nmax = 0;
#pragma unroll
        for (int u = 0; u < CG_SROWS; ++u) {
            const int64_t iu = i + (int64_t)u * CG_WAVES;
            has[u] = iu < r1;
            const int64_t ic = has[u] ? iu : i;
            e0[u] = rowptr[ic];
            ne[u] = rowptr[ic + 1] - e0[u];
            nmax = ne[u] > nmax ? ne[u] : nmax;
            o[u] = ic * k + jj;
            zo[u] = zval<V>(dinv[ic], R[o[u]]);
            po[u] = fresh ? 0.0 : (double)P[o[u]];
            qo[u] = fresh ? 0.0 : (double)Q[o[u]];
            acc[u] = 0.0;
        }
        for (int64_t e = 0; e < nmax; e += CG_GATHER) {
            V rg[CG_SROWS][CG_GATHER];
            double vg[CG_SROWS][CG_GATHER];
#pragma unroll
            for (int u = 0; u < CG_SROWS; ++u)
#pragma unroll
                for (int g = 0; g < CG_GATHER; ++g) {
                    const bool in = e + g < ne[u];
                    const int64_t x = in ? e0[u] + e + g : e0[u] + ne[u] - 1;
                    vg[u][g] = in ? vd[x] : 0.0;
                    rg[u][g] = R[(int64_t)col[x] * k + jj];
                }
#pragma unroll
            for (int u = 0; u < CG_SROWS; ++u)
#pragma unroll
                for (int g = 0; g < CG_GATHER; ++g) acc[u] += vg[u][g] * (double)rg[u][g];
        }
        if (jok) {
#pragma unroll
            for (int u = 0; u < CG_SROWS; ++u) {
                if (!has[u]) continue;
                const V pn = (V)(fresh ? zo[u] : zo[u] + beta * po[u]);
                const V qn = (V)(fresh ? acc[u] : acc[u] + beta * qo[u]);
                P[o[u]] = pn;
                Q[o[u]] = qn;
                pq += (double)pn * (double)qn;
            }
        }
    }
    __shared__ double red[CG_WAVES][64];
    red[wave][lane] = pq;
    __syncthreads();
    if (wave == 0) {
        double s = 0.0;
        for (int w = 0; w < CG_WAVES; ++w) s += red[w][lane];
        if (jok) part[(int64_t)ty * k + j] = s;
    }
}

template <typename V>
__global__ __launch_bounds__(CG_THREADS) void k_cg_update(
    int64_t n, int k, const double* __restrict__ dinv, double* __restrict__ W,
    V* __restrict__ R, const V* __restrict__ P, const V* __restrict__ Q,
    const double* __restrict__ scal, const double* __restrict__ pqp, double* __restrict__ part,
    int* __restrict__ tctl, int* __restrict__ mctl, int it, int gx, int gy, int64_t rows_per,
    int mode) {
    const Tile T = cg_tile(mode, gx, gy);
    if (!T.ok) return;
    const int tx = T.tx, ty = T.ty;
    if (tctl[tx * T_INTS + T_DONE]) return;
    const int lane = threadIdx.x & 63;
    const int wave = wave_id();
    const int j = tx * 64 + lane;
    const bool jok = j < k;
    const int jj = jok ? j : k - 1;
    // alpha = r.z / p.q (p.q summed in a fixed order, as in the product's prologue)
    __shared__ double psum[CG_WAVES][64];
    double pv[CG_TPW];
#pragma unroll
    for (int u = 0; u < CG_TPW; ++u) {
        const int t = wave + CG_WAVES * u;
        pv[u] = pqp[(int64_t)(t < gy ? t : 0) * k + jj];
    }
    double a = 0.0;
#pragma unroll
    for (int u = 0; u < CG_TPW; ++u)
        if (wave + CG_WAVES * u < gy) a += pv[u];
    psum[wave][lane] = a;
    __syncthreads();
    double pq = 0.0;
    for (int w = 0; w < CG_WAVES; ++w) pq += psum[w][lane];
    const double rz0 = scal[jj * 4 + (it & 1)];
    const double alpha = (jok && pq > 0.0 && rz0 > 0.0) ? rz0 / pq : 0.0;
    // breakdown: a non-zero residual whose direction has p.Ap <= 0 (every
    // workgroup of the tile sees the same sums; row tile 0 records it)
    const bool bad = jok && rz0 > 0.0 && !(pq > 0.0);
    if (__any(bad)) {
        if (ty == 0 && wave == 0 && lane == 0) {
            int* c = tctl + tx * T_INTS;
            c[T_BAD] = 1;
            c[T_DONE] = 1;
            if (mctl) {
                mctl[tx * T_INTS + T_BAD] = 1;
                mctl[tx * T_INTS + T_DONE] = 1;
            }
        }
        return;
    }
    double rz = 0.0, rr = 0.0;
    const int64_t r0 = (int64_t)ty * rows_per;
    const int64_t r1 = r0 + rows_per < n ? r0 + rows_per : n;
    if (jok) {
        // CG_UROWS rows per wave at a time (i, i + 8, ...): all their loads in
        // flight before the first store; missing rows repeat row i, unstored
        for (int64_t i = r0 + wave; i < r1; i += CG_UROWS * CG_WAVES) {
            int64_t o[CG_UROWS];
            bool has[CG_UROWS];
            double wv[CG_UROWS], pv[CG_UROWS], rv[CG_UROWS], qv[CG_UROWS], dv[CG_UROWS];
#pragma unroll
            for (int u = 0; u < CG_UROWS; ++u) {
                const int64_t iu = i + (int64_t)u * CG_WAVES;
                has[u] = iu < r1;
                const int64_t ic = has[u] ? iu : i;
                o[u] = ic * k + j;
                wv[u] = W[o[u]];
                pv[u] = (double)P[o[u]];
                rv[u] = (double)R[o[u]];
                qv[u] = (double)Q[o[u]];
                dv[u] = dinv[ic];
            }
#pragma unroll
            for (int u = 0; u < CG_UROWS; ++u) {
                if (!has[u]) continue;
                W[o[u]] = wv[u] + alpha * pv[u];
                const V rn = (V)(rv[u] - alpha * qv[u]);
                R[o[u]] = rn;
                const double zn = zval<V>(dv[u], rn);
                rz += (double)rn * zn;
                rr += (double)rn * (double)rn;
            }
        }
    }
    __shared__ double red[2][CG_WAVES][64];
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
            part[((int64_t)ty * k + j) * 2 + 0] = s0;
            part[((int64_t)ty * k + j) * 2 + 1] = s1;
        }
    }
}

// Residual replacement for float vectors: r = e_j - A x from the float64
// iterate x (W), in float64, with the same partial sums as the update. The
// recursively updated float residual drifts from the true one; replacing it
// every few iterations keeps the convergence test honest.
template <typename V>
__global__ __launch_bounds__(CG_THREADS) void k_cg_true_residual(
    const int64_t* __restrict__ rowptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, int64_t n, int k, const int32_t* __restrict__ cols,
    const double* __restrict__ dinv, const double* __restrict__ W, V* __restrict__ R,
    double* __restrict__ part, const int* __restrict__ tctl, int gx, int gy, int64_t rows_per,
    int mode) {
    const Tile T = cg_tile(mode, gx, gy);
    if (!T.ok) return;
    const int tx = T.tx, ty = T.ty;
    if (tctl[tx * T_INTS + T_DONE]) return;
    const int lane = threadIdx.x & 63;
    const int wave = wave_id();
    const int j = tx * 64 + lane;
    const bool jok = j < k;
    const int jj = jok ? j : k - 1;
    const int64_t cj = cols[jj];
    double rz = 0.0, rr = 0.0;
    const int64_t r0 = (int64_t)ty * rows_per;
    const int64_t r1 = r0 + rows_per < n ? r0 + rows_per : n;
    for (int64_t i = r0 + wave; i < r1; i += CG_WAVES) {
        const int64_t e0 = rowptr[i], ne = rowptr[i + 1] - e0;
        double acc = 0.0;
        // gathers in batches of 8, all issued together; a short batch repeats
        // the row's last entry with a zero coefficient (adds +0: the sum is the
        // entry-by-entry one)
        for (int64_t e = 0; e < ne; e += 8) {
            double wv[8], av[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const bool in = e + u < ne;
                const int64_t x = in ? e0 + e + u : e0 + ne - 1;
                av[u] = in ? val[x] : 0.0;
                wv[u] = W[(int64_t)col[x] * k + jj];
            }
#pragma unroll
            for (int u = 0; u < 8; ++u) acc += av[u] * wv[u];
        }
        if (jok) {
            const int64_t o = i * k + j;
            const double r = (i == cj ? 1.0 : 0.0) - acc;
            const V rv = (V)r;
            R[o] = rv;
            const double zv = zval<V>(dinv[i], rv);
            rz += (double)rv * zv;
            rr += (double)rv * (double)rv;
        }
    }
    __shared__ double red[2][CG_WAVES][64];
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
            part[((int64_t)ty * k + j) * 2 + 0] = s0;
            part[((int64_t)ty * k + j) * 2 + 1] = s1;
        }
    }
}

}  // namespace

namespace {

constexpr int CG_REPLACE_EVERY = 8;   // float vectors: true residual every this many iterations

// The sparse matrix as raw device pointers (the solver's CSR, or a caller's).
struct CsrView {
    const int64_t* rowptr;
    const int32_t* col;
    const double* val;
    int64_t n, nnz;
};

// Buffers of one solve. Device: dinv (n), vd (nnz), part (row_tiles * k * 3), scal
// (4k + col_tiles), flags (T_INTS * col_tiles). Host: hctl (T_INTS *
// col_tiles ints) and hres (col_tiles doubles), the host's view of the control
// words. mirror: hctl and hres are pinned, and the kernels write them beside
// the device words (a check then copies nothing); otherwise each check copies
// them. predicted: iterations of the last solve of this kind (read and
// updated). prof: record launches with the profiler.
struct CGBufs {
    double* dinv;
    double* vd;
    double* part;
    double* scal;
    int* flags;
    int* hctl;
    double* hres;
    int* predicted;
    bool prof;
    bool mirror;
};

// Launch geometry of one solve: gx 64-column tiles; gy row tiles of rows_per
// contiguous rows (each wave takes at least two rows); the tile mapping mode
// of cg_tile (column-grouped with 8 or more column tiles, else row-banded when
// there are 8 or more row tiles) and its grid.
struct CgGeom {
    int gx, gy, mode;
    int64_t rows_per;
    dim3 grid;
};

CgGeom cg_geom(int64_t n, int k) {
    CgGeom g;
    g.gx = (std::max(k, 1) + 63) / 64;
    int gy = (int)std::min<int64_t>(CG_ROW_TILES, (n + 2 * CG_WAVES - 1) / (2 * CG_WAVES));
    if (gy < 1) gy = 1;
    if (g.gx >= 8) {
        g.mode = 1;
        g.gy = gy;
        g.grid = dim3((unsigned)(8 * ((g.gx + 7) / 8) * gy));
    } else if (gy >= 8) {
        g.mode = 2;
        g.gy = gy / 8 * 8;
        g.grid = dim3((unsigned)(g.gx * g.gy));
    } else {
        g.mode = 0;
        g.gy = gy;
        g.grid = dim3((unsigned)g.gx, (unsigned)gy);
    }
    g.rows_per = (n + g.gy - 1) / g.gy;
    return g;
}

int cg_row_tiles(int64_t n, int k) { return cg_geom(n, k).gy; }

template <typename V>
CGResult block_cg_impl(const CsrView& A, const int32_t* d_cols, int k, double* W, double tol,
                       int max_iter, const CGBufs& bf, V* R, V* P, V* Q, hipStream_t s,
                       const WarmStore* ws = nullptr) {
    constexpr bool LOW = sizeof(V) < sizeof(double);
    CGResult res;
    const int64_t n = A.n;
    if (k <= 0) {
        res.converged = true;
        return res;
    }
    const CgGeom G = cg_geom(n, k);
    const bool wide = A.nnz > (int64_t)CG_WIDE_ROW * n;
    int* hm_ctl = bf.mirror ? bf.hctl : nullptr;   // host mirrors of the control words
    double* hm_res = bf.mirror ? bf.hres : nullptr;
    const int col_tiles = G.gx;
    const int row_tiles = G.gy;
    // partials: r.z and r.r of an update (two per entry), then p.q of a product
    double* part_rz = bf.part;
    double* part_pq = bf.part + (size_t)row_tiles * k * 2;
    double* tres = bf.scal + 4 * k;
    hipLaunchKernelGGL(k_cg_dinv, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       A.rowptr, A.col, A.val, n, bf.dinv);
    SIC_CHECK_LAUNCH();
    hipLaunchKernelGGL(k_cg_vd, dim3((unsigned)std::min<int64_t>((A.nnz + 255) / 256, 4096)),
                       dim3(256), 0, s, A.col, A.val, bf.dinv, A.nnz, bf.vd);
    SIC_CHECK_LAUNCH();
    // (with a warm start, init only clears the control words: x0 and r0 come next)
    hipLaunchKernelGGL(k_cg_init<V>, dim3(ws ? 1u : (unsigned)std::min<int64_t>(n, 4096)), dim3(256),
                       0, s, n, k, col_tiles, d_cols, bf.dinv, W, R, bf.scal, bf.flags, tres,
                       hm_ctl, hm_res, ws ? 0 : 1);
    SIC_CHECK_LAUNCH();
    // warm start: x0 from the store, r0 = e - A x0 exactly, and the iterations
    // begin at 1, the first product starting p and q from zero
    int start = 0;
    if (ws) {
        const dim3 tg((unsigned)((k + 63) / 64), (unsigned)((n + 63) / 64));
        hipLaunchKernelGGL(k_cg_warm, tg, dim3(256), 0, s, n, k, d_cols, ws->W, ws->valid, W);
        SIC_CHECK_LAUNCH();
        hipLaunchKernelGGL(k_cg_true_residual<V>, G.grid, dim3(CG_THREADS), 0, s, A.rowptr, A.col,
                           A.val, n, k, d_cols, bf.dinv, W, R, part_rz, bf.flags, col_tiles,
                           row_tiles, G.rows_per, G.mode);
        SIC_CHECK_LAUNCH();
        start = 1;
    }
    const int* hctl = bf.hctl;
    const double* hres = bf.hres;
    int& predicted = *bf.predicted;
    int launched = start;
    int active = col_tiles;   // tiles still iterating (as of the last check)
    // algorithmic traffic of one tile-launch (bytes): the sparse matrix once,
    // each n x 64 block touched once per read or write
    const double mat = (double)A.nnz * 12.0 + (double)(n + 1) * 8.0;
    struct Rec {
        int64_t spmm, upd;
        int iter;
    };
    std::vector<Rec> recs;
    bool done = false;
    while (launched < max_iter && !done) {
        // the first check where the last solve of this kind converged (its last
        // update is tested by the next launch's product), then every 4 or 8
        const int first = predicted > 0 ? predicted + 1 : 4;
        const int chunk = std::min(launched == start ? first : (launched < 16 ? 4 : 8),
                                   max_iter - launched);
        recs.clear();
        for (int c = 0; c < chunk; ++c) {
            const int it = launched + c;
            const double nkb = (double)n * k * sizeof(V);
            Rec r;
            r.iter = it;
            if (bf.prof) prof_begin(KK_CG_SPMM, s);
            if (wide)
                hipLaunchKernelGGL((k_cg_spmm<V, 16>), G.grid, dim3(CG_THREADS), 0, s, A.rowptr,
                                   A.col, bf.vd, n, k, bf.dinv, R, P, Q, bf.scal, part_rz,
                                   part_pq, bf.flags, tres, hm_ctl, hm_res, tol, it, start,
                                   col_tiles, row_tiles, G.rows_per, G.mode, 0);
            else
                hipLaunchKernelGGL((k_cg_spmm<V, 8>), G.grid, dim3(CG_THREADS), 0, s, A.rowptr,
                                   A.col, bf.vd, n, k, bf.dinv, R, P, Q, bf.scal, part_rz,
                                   part_pq, bf.flags, tres, hm_ctl, hm_res, tol, it, start,
                                   col_tiles, row_tiles, G.rows_per, G.mode, 0);
            SIC_CHECK_LAUNCH();
            if (bf.prof)
                r.spmm = prof_end(KK_CG_SPMM, s, mat + (it == 0 ? 3.0 : 5.0) * nkb,
                                  2.0 * A.nnz * k + 4.0 * n * k);
            if (bf.prof) prof_begin(KK_CG_UPDATE, s);
            hipLaunchKernelGGL(k_cg_update<V>, G.grid, dim3(CG_THREADS), 0, s, n, k, bf.dinv, W,
                               R, P, Q, bf.scal, part_pq, part_rz, bf.flags, hm_ctl, it, col_tiles,
                               row_tiles, G.rows_per, G.mode);
            SIC_CHECK_LAUNCH();
            if (bf.prof)
                r.upd = prof_end(KK_CG_UPDATE, s, 4.0 * nkb + 16.0 * n * k + n * 8.0,
                                 10.0 * n * k);
            if (LOW && (it + 1) % CG_REPLACE_EVERY == 0) {
                hipLaunchKernelGGL(k_cg_true_residual<V>, G.grid, dim3(CG_THREADS), 0, s,
                                   A.rowptr, A.col, A.val, n, k, d_cols, bf.dinv, W, R, part_rz,
                                   bf.flags, col_tiles, row_tiles, G.rows_per, G.mode);
                SIC_CHECK_LAUNCH();
            }
            if (bf.prof) recs.push_back(r);
        }
        launched += chunk;
        if (launched >= max_iter) {
            // the last update's residual has no product after it to test it
            hipLaunchKernelGGL((k_cg_spmm<V, 8>), dim3(col_tiles, 1), dim3(CG_THREADS), 0, s,
                               A.rowptr, A.col, bf.vd, n, k, bf.dinv, R, P, Q, bf.scal, part_rz,
                               part_pq, bf.flags, tres, hm_ctl, hm_res, tol, launched, start,
                               col_tiles, row_tiles, G.rows_per, 0, 1);
            SIC_CHECK_LAUNCH();
        }
        if (!bf.mirror) {
            SIC_HIP(hipMemcpyAsync(bf.hctl, bf.flags, sizeof(int) * T_INTS * col_tiles,
                                   hipMemcpyDeviceToHost, s));
            SIC_HIP(hipMemcpyAsync(bf.hres, tres, sizeof(double) * col_tiles,
                                   hipMemcpyDeviceToHost, s));
        }
        stream_wait(s);
        // a launch did work only for the tiles still iterating at its index:
        // scale its algorithmic bytes, drop launches that found nothing to do
        for (const Rec& r : recs) {
            int working = 0;
            for (int t = 0; t < col_tiles; ++t) working += hctl[t * T_INTS + T_ITER] > r.iter;
            if (working == 0) {
                prof_discard(r.spmm);
                prof_discard(r.upd);
            } else if (working < col_tiles) {
                prof_scale(r.spmm, (double)working / col_tiles);
                prof_scale(r.upd, (double)working / col_tiles);
            }
        }
        done = true;
        active = 0;
        for (int t = 0; t < col_tiles; ++t)
            if (!hctl[t * T_INTS + T_DONE]) {
                done = false;
                ++active;
            }
    }
    (void)active;
    if (bf.prof) prof_flush();
    int iters = 0;
    double mres = 0.0;
    bool bad = false;
    for (int t = 0; t < col_tiles; ++t) {
        iters = std::max(iters, hctl[t * T_INTS + T_ITER]);
        mres = std::max(mres, hres[t]);
        bad = bad || hctl[t * T_INTS + T_BAD] != 0;
    }
    res.iterations = iters;
    res.breakdown = bad;
    res.converged = done && !bad;
    res.max_rel_res = mres;
    predicted = res.converged ? iters : 0;
    if (ws && res.converged) {
        const dim3 tg((unsigned)((k + 63) / 64), (unsigned)((n + 63) / 64));
        hipLaunchKernelGGL(k_cg_store, tg, dim3(256), 0, s, n, k, d_cols, W, ws->W, ws->valid);
        SIC_CHECK_LAUNCH();
    }
    return res;
}

}  // namespace

void check_cg(const CGResult& r, const char* what) {
    if (r.breakdown)
        throw SicError(SIC_ENOTPD, std::string(what) +
                                       ": conjugate gradients broke down (p.Ap <= 0), the iterate "
                                       "is not positive definite");
    if (!r.converged)
        throw SicError(SIC_ENOCONV, std::string(what) + ": conjugate gradients did not reach "
                                                        "their tolerance within cg_max_iter");
}

CGResult block_cg(const DevCSR& A, const int32_t* d_cols, int k, double* W, int64_t ldw,
                  double tol, int max_iter, CGWork& wk, hipStream_t s, bool low_precision,
                  int slot, const WarmStore* ws) {
    if (k > 0 && ldw != k) throw SicError(SIC_EINTERNAL, "block_cg expects ldw == k");
    const int64_t n = A.n;
    const size_t nk = (size_t)n * (size_t)std::max(k, 1);
    const int col_tiles = (std::max(k, 1) + 63) / 64;
    wk.dinv.reserve(n);
    wk.vd.reserve((size_t)std::max<int64_t>(A.nnz, 1));
    wk.part.reserve((size_t)cg_row_tiles(n, k) * std::max(k, 1) * 3);
    wk.scal.reserve((size_t)4 * std::max(k, 1) + col_tiles);
    wk.flags.reserve((size_t)T_INTS * col_tiles);
    wk.hctl.reserve((size_t)T_INTS * col_tiles);
    wk.hres.reserve(col_tiles);
    const CsrView av{A.rowptr.p, A.col.p, A.val.p, A.n, A.nnz};
    CGBufs bf{wk.dinv.p, wk.vd.p, wk.part.p, wk.scal.p, wk.flags.p, wk.hctl.p, wk.hres.p,
              &wk.predict[(slot & 3) * 2 + (low_precision ? 1 : 0)], true, true};
    if (low_precision) {
        wk.R32.reserve(nk);
        wk.P32.reserve(nk);
        wk.Q32.reserve(nk);
        return block_cg_impl<float>(av, d_cols, k, W, tol, max_iter, bf, wk.R32.p, wk.P32.p,
                                    wk.Q32.p, s, ws);
    }
    wk.R.reserve(nk);
    wk.P.reserve(nk);
    wk.Q.reserve(nk);
    return block_cg_impl<double>(av, d_cols, k, W, tol, max_iter, bf, wk.R.p, wk.P.p, wk.Q.p,
                                 s, ws);
}

// ------------------------------------------------------------------------
// Inverse columns with no allocation: every buffer of the solve lives in one
// file-scope device array (per GPU, for the life of the process). The host
// names the array only through the address hipGetSymbolAddress gives for the
// current device; the kernels take that address like any other buffer.

namespace {

constexpr size_t NOALLOC_SCRATCH_BYTES = (size_t)128 << 20;
constexpr int NOALLOC_MAX_K = 4096;
constexpr int NOALLOC_MAX_TILES = NOALLOC_MAX_K / 64;
constexpr int NOALLOC_MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

std::mutex g_scratch_mu;
void* g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

size_t align256(size_t x) { return (x + 255) & ~(size_t)255; }

// Device address of this GPU's scratch array (looked up once per device).
unsigned char* scratch_address() {
    int dev = 0;
    SIC_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES)
        throw SicError(SIC_EINVAL, "device ordinal out of range");
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        SIC_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_scratch_ptr[dev] = p;
    }
    return static_cast<unsigned char*>(g_scratch_ptr[dev]);
}

}  // namespace

size_t cg_noalloc_bytes(int64_t n, int64_t nnz, int k) {
    const int ct = (k + 63) / 64;
    return align256(sizeof(double) * (size_t)n) + align256(sizeof(double) * (size_t)nnz) +
           align256(sizeof(double) * (size_t)cg_row_tiles(n, k) * k * 3) +
           align256(sizeof(double) * ((size_t)4 * k + ct)) + align256(sizeof(int) * T_INTS * ct) +
           3 * align256(sizeof(double) * (size_t)n * k);
}

size_t cg_noalloc_capacity() { return NOALLOC_SCRATCH_BYTES; }
int cg_noalloc_max_k() { return NOALLOC_MAX_K; }

CGResult block_cg_noalloc(const int64_t* rowptr, const int32_t* col, const double* val,
                          int64_t n, int64_t nnz, const int32_t* d_cols, int k, double* W,
                          double tol, int max_iter, hipStream_t s) {
    if (k > NOALLOC_MAX_K || cg_noalloc_bytes(n, nnz, k) > NOALLOC_SCRATCH_BYTES)
        throw SicError(SIC_ETOOBIG, "inverse columns without allocation: n x k = " +
                                        std::to_string(n) + " x " + std::to_string(k) +
                                        " needs " + std::to_string(cg_noalloc_bytes(n, nnz, k)) +
                                        " bytes of scratch, the limit is " +
                                        std::to_string(NOALLOC_SCRATCH_BYTES) +
                                        " (and k <= " + std::to_string(NOALLOC_MAX_K) + ")");
    unsigned char* base = scratch_address();
    const int ct = (k + 63) / 64;
    size_t off = 0;
    auto take = [&](size_t bytes) {
        unsigned char* p = base + off;
        off += align256(bytes);
        return p;
    };
    double* dinv = reinterpret_cast<double*>(take(sizeof(double) * (size_t)n));
    double* vd = reinterpret_cast<double*>(take(sizeof(double) * (size_t)nnz));
    double* part =
        reinterpret_cast<double*>(take(sizeof(double) * (size_t)cg_row_tiles(n, k) * k * 3));
    double* scal = reinterpret_cast<double*>(take(sizeof(double) * ((size_t)4 * k + ct)));
    int* flags = reinterpret_cast<int*>(take(sizeof(int) * T_INTS * ct));
    const size_t nkb = sizeof(double) * (size_t)n * k;
    double* R = reinterpret_cast<double*>(take(nkb));
    double* P = reinterpret_cast<double*>(take(nkb));
    double* Q = reinterpret_cast<double*>(take(nkb));
    // control read-backs land in host stack arrays (pageable copies)
    int hctl[T_INTS * NOALLOC_MAX_TILES];
    double hres[NOALLOC_MAX_TILES];
    int predicted = 0;
    const CsrView av{rowptr, col, val, n, nnz};
    const CGBufs bf{dinv, vd, part, scal, flags, hctl, hres, &predicted, false, false};
    return block_cg_impl<double>(av, d_cols, k, W, tol, max_iter, bf, R, P, Q, s);
}

}  // namespace sic
