// Small device utilities: single-workgroup prefix scans and index helpers
// used to compact free sets, neighbourhoods and CSR rows in a fixed order.
#include "sic_internal.h"

namespace sic {

namespace {

constexpr int SCAN_THREADS = 1024;

// Exclusive scan of `count` int32 values into int64 (out has count+1 entries,
// out[count] = total). One workgroup; each thread owns a contiguous chunk.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_i32(const int32_t* __restrict__ in,
                                                           int64_t count, int64_t* __restrict__ out,
                                                           int64_t* __restrict__ total_out) {
    __shared__ int64_t sums[SCAN_THREADS];
    const int t = threadIdx.x;
    const int64_t chunk = (count + SCAN_THREADS - 1) / SCAN_THREADS;
    const int64_t b0 = t * chunk, b1 = b0 + chunk < count ? b0 + chunk : count;
    constexpr int G = 8;   // eight loads in flight per batch (clamped past the chunk end)
    int64_t s = 0;
    for (int64_t i0 = b0; i0 < b1; i0 += G) {
        int32_t v[G];
#pragma unroll
        for (int u = 0; u < G; ++u) v[u] = in[i0 + u < b1 ? i0 + u : b0];
#pragma unroll
        for (int u = 0; u < G; ++u)
            if (i0 + u < b1) s += v[u];
    }
    sums[t] = s;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        int64_t v = t >= off ? sums[t - off] : 0;
        __syncthreads();
        sums[t] += v;
        __syncthreads();
    }
    int64_t run = t > 0 ? sums[t - 1] : 0;
    for (int64_t i0 = b0; i0 < b1; i0 += G) {
        int32_t v[G];
#pragma unroll
        for (int u = 0; u < G; ++u) v[u] = in[i0 + u < b1 ? i0 + u : b0];
#pragma unroll
        for (int u = 0; u < G; ++u) {
            if (i0 + u >= b1) break;
            out[i0 + u] = run;
            run += v[u];
        }
    }
    if (t == SCAN_THREADS - 1) {
        out[count] = sums[t];
        if (total_out) *total_out = sums[t];
    }
}

// Scan of per-(tile, column) counts in column-major order (column outer,
// tile inner): offsets[tile*b + c] = number of entries of columns < c plus
// entries of column c in tiles < tile. colptr[c] = offsets[0*b + c], and
// colptr[b] the total. b <= 256: thread t takes column t % 256 over a quarter
// of the tiles (group t / 256), so every load reads a contiguous row segment
// of the count matrix: column sums by quarter, an exclusive scan of the column
// totals, then the offsets in a second pass.
constexpr int CM_COLS = 256;
constexpr int CM_GROUPS = SCAN_THREADS / CM_COLS;

__global__ __launch_bounds__(SCAN_THREADS) void k_scan_colmajor(const int32_t* __restrict__ cnt,
                                                                int tiles, int b,
                                                                int32_t* __restrict__ offsets,
                                                                int64_t* __restrict__ colptr,
                                                                int64_t* __restrict__ total) {
    __shared__ int64_t part[CM_GROUPS][CM_COLS];
    __shared__ int64_t cs[CM_COLS];
    const int t = threadIdx.x;
    const int c = t % CM_COLS, g = t / CM_COLS;
    const bool on = c < b;
    const int tile0 = (int)((int64_t)g * tiles / CM_GROUPS);
    const int tile1 = (int)((int64_t)(g + 1) * tiles / CM_GROUPS);
    constexpr int G = 8;   // loads in flight per batch, clamped to a valid entry
    auto gather = [&](int q0, int32_t* v) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int tile = q0 + u < tile1 ? q0 + u : tile0;
            v[u] = cnt[(int64_t)tile * b + (on ? c : 0)];
        }
    };
    int64_t s = 0;
    for (int q0 = tile0; q0 < tile1; q0 += G) {
        int32_t v[G];
        gather(q0, v);
#pragma unroll
        for (int u = 0; u < G; ++u)
            if (q0 + u < tile1) s += v[u];
    }
    part[g][c] = on ? s : 0;
    __syncthreads();
    // column totals, then their inclusive scan over the columns (group 0)
    if (g == 0) {
        int64_t tot = 0;
        for (int q = 0; q < CM_GROUPS; ++q) tot += part[q][c];
        cs[c] = tot;
    }
    __syncthreads();
    for (int off = 1; off < CM_COLS; off <<= 1) {
        const int64_t v = (g == 0 && c >= off) ? cs[c - off] : 0;
        __syncthreads();
        if (g == 0) cs[c] += v;
        __syncthreads();
    }
    // this thread's start: entries of columns < c, then of column c in earlier quarters
    int64_t run = c > 0 ? cs[c - 1] : 0;
    for (int q = 0; q < g; ++q) run += part[q][c];
    if (g == 0 && on) colptr[c] = run;
    if (t == 0) {
        colptr[b] = cs[b - 1];
        if (total) *total = cs[b - 1];
    }
    for (int q0 = tile0; q0 < tile1; q0 += G) {
        int32_t v[G];
        gather(q0, v);
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int tile = q0 + u;
            if (tile < tile1 && on) {
                offsets[(int64_t)tile * b + c] = (int32_t)run;
                run += v[u];
            }
        }
    }
}

__global__ void k_fill_i32(int32_t* __restrict__ p, int64_t count, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = v;
}

__global__ void k_iota_i32(int32_t* __restrict__ p, int64_t count, int32_t start) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) p[i] = start + (int32_t)i;
}

}  // namespace

void launch_scan_i32(const int32_t* in, int64_t count, int64_t* out, int64_t* total, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_i32, dim3(1), dim3(SCAN_THREADS), 0, s, in, count, out, total);
    SIC_CHECK_LAUNCH();
}

void launch_scan_colmajor(const int32_t* cnt, int tiles, int b, int32_t* offsets, int64_t* colptr,
                          int64_t* total, hipStream_t s) {
    if (b < 1 || b > CM_COLS || tiles < 1)
        throw SicError(SIC_EINTERNAL, "column-major scan: 1 <= b <= 256 and tiles >= 1 required");
    hipLaunchKernelGGL(k_scan_colmajor, dim3(1), dim3(SCAN_THREADS), 0, s, cnt, tiles, b, offsets,
                       colptr, total);
    SIC_CHECK_LAUNCH();
}

void launch_fill_i32(int32_t* p, int64_t count, int32_t v, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, v);
    SIC_CHECK_LAUNCH();
}

namespace {
__global__ void k_gather_cols(const double* __restrict__ X, int64_t m, int64_t n,
                              const int32_t* __restrict__ perm, double* __restrict__ out) {
    // one row of samples per workgroup step; the row's gathers stay in one
    // 8n-byte segment
    for (int64_t r = blockIdx.y; r < m; r += gridDim.y) {
        const double* xr = X + r * n;
        double* orow = out + r * n;
        for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
             c += (int64_t)gridDim.x * blockDim.x)
            orow[c] = xr[perm[c]];
    }
}
}  // namespace

void launch_gather_cols(const double* X, int64_t m, int64_t n, const int32_t* perm, double* out,
                        hipStream_t s) {
    if (m <= 0 || n <= 0) return;
    const unsigned gx = (unsigned)std::min<int64_t>((n + 255) / 256, 64);
    const unsigned gy = (unsigned)std::min<int64_t>(m, 1024);
    hipLaunchKernelGGL(k_gather_cols, dim3(gx, gy), dim3(256), 0, s, X, m, n, perm, out);
    SIC_CHECK_LAUNCH();
}

void launch_iota_i32(int32_t* p, int64_t count, int32_t start, hipStream_t s) {
    if (count <= 0) return;
    hipLaunchKernelGGL(k_iota_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count,
                       start);
    SIC_CHECK_LAUNCH();
}


namespace {
__global__ void k_coord_globals(int64_t nc, const int32_t* __restrict__ c_p,
                                const int32_t* __restrict__ c_ci, const int32_t* __restrict__ Jp,
                                int64_t j0, int32_t* __restrict__ gr, int32_t* __restrict__ gc) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nc) return;
    gr[t] = Jp[c_p[t]];
    gc[t] = (int32_t)(j0 + c_ci[t]);
}
}  // namespace

void launch_coord_globals(int64_t nc, const int32_t* c_p, const int32_t* c_ci, const int32_t* Jp,
                          int64_t j0, int32_t* gr, int32_t* gc, hipStream_t s) {
    if (nc <= 0) return;
    hipLaunchKernelGGL(k_coord_globals, dim3((unsigned)((nc + 255) / 256)), dim3(256), 0, s, nc,
                       c_p, c_ci, Jp, j0, gr, gc);
    SIC_CHECK_LAUNCH();
}

}  // namespace sic
