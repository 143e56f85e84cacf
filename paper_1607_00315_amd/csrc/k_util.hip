// Small device utilities: single-workgroup prefix scans and index helpers
// used to compact free sets, neighbourhoods and CSR rows in a fixed order.
#include "sic_internal.h"

namespace sic {

namespace {

constexpr int SCAN_THREADS = 1024;
constexpr int SCAN_WAVES = SCAN_THREADS / 64;

// Inclusive scan of one value per lane across a 64-lane wavefront.
__device__ inline int64_t wave_inclusive_scan(int64_t x, int lane) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const long long y = __shfl_up((long long)x, off, 64);
        if (lane >= off) x += y;
    }
    return x;
}

// Exclusive scan of `count` int32 values into int64 (out has count+1 entries,
// out[count] = total). One workgroup; each thread owns a contiguous chunk.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_i32(const int32_t* __restrict__ in,
                                                           int64_t count, int64_t* __restrict__ out,
                                                           int64_t* __restrict__ total_out) {
    __shared__ int64_t wsum[SCAN_WAVES];
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
    // chunk sums: inclusive scan within each wavefront, then over the wave totals
    const int lane = t & 63, w = t >> 6;
    const int64_t inc = wave_inclusive_scan(s, lane);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    if (w == 0) {
        const int64_t x = wave_inclusive_scan(lane < SCAN_WAVES ? wsum[lane] : 0, lane);
        if (lane < SCAN_WAVES) wsum[lane] = x;
    }
    __syncthreads();
    int64_t run = inc - s + (w > 0 ? wsum[w - 1] : 0);
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
    if (t == 0) {
        out[count] = wsum[SCAN_WAVES - 1];
        if (total_out) *total_out = wsum[SCAN_WAVES - 1];
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
    __shared__ int64_t cw[CM_COLS / 64];
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
    // column totals (group 0), scanned within each wavefront of 64 columns;
    // the exclusive in-wave prefix of every column and the wave totals go to LDS
    if (g == 0) {
        int64_t tot = 0;
        for (int q = 0; q < CM_GROUPS; ++q) tot += part[q][c];
        const int64_t inc = wave_inclusive_scan(tot, c & 63);
        cs[c] = inc - tot;
        if ((c & 63) == 63) cw[c >> 6] = inc;
    }
    __syncthreads();
    // this thread's start: entries of columns < c, then of column c in earlier quarters
    int64_t run = cs[c];
    for (int q = 0; q < (c >> 6); ++q) run += cw[q];
    for (int q = 0; q < g; ++q) run += part[q][c];
    if (g == 0 && on) colptr[c] = run;
    if (t == 0) {
        int64_t all = 0;
        for (int q = 0; q < CM_COLS / 64; ++q) all += cw[q];
        colptr[b] = all;
        if (total) *total = all;
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
