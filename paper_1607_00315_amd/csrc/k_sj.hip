// Covariance columns from the samples (Section 6: the samples are stored, S is
// never formed; the trace term costs O(nnz * m), Section 6.1.2).
//
//   S_J = X^T X[:, J] / m      (n x b, dense, finest level)
//   S_rc = X[:, r] . X[:, c] / m  for listed pairs (coarse levels, Section 7:
//                                  only the entries of C_l are needed)
//
// X is m x n row-major float64.  The dense block is an MFMA contraction over
// the m samples (v_mfma_f64_16x16x4f64); sampled entries are wave-wide dot
// products over rows of the transposed copy Xt (n x m row-major).
#include "profiler.h"

#include <type_traits>

namespace sic {

typedef double double4_t __attribute__((ext_vector_type(4)));

namespace {

constexpr int SJ_TILE = 64;   // output tile: 64 rows of S_J x 64 block columns
constexpr int SJ_KC = 16;     // samples staged per LDS round
constexpr int SJ_PAD = 4;

// One workgroup = 4 waves = one 64 x 64 output tile; wave (wr, wc) owns a
// 32 x 32 quadrant as 2 x 2 MFMA 16x16 accumulators.
// MFMA f64 16x16x4 operand layout: lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; the 16x16 result sits in 4 registers per lane as
// D[(l/16) + 4*v][l%16], v = 0..3 (checked with a lane-layout probe).
// Tile order: a 1-D grid whose workgroup L runs on XCD L % 8 (round-robin
// dispatch). Each XCD takes every eighth 64-row slab and runs the slab's
// column tiles one after another, so the slab of X they all read is fetched
// into that XCD's L2 once instead of once per column tile.
// ks (1 or 2) splits the samples of every tile between ks workgroups (the
// grid has 2.5 tiles per compute unit otherwise, unevenly spread). With two,
// both halves are added atomically into the zeroed output: 0 + a + b is a + b
// exactly in either order, so the result does not depend on which lands first.
__global__ __launch_bounds__(256) void k_sj_gemm_f64(const double* __restrict__ X, int64_t n,
                                                     int64_t m, int64_t j0, int b,
                                                     double* __restrict__ out, double invm,
                                                     int row_tiles, int col_tiles, int ks) {
    // two LDS buffers by round parity: the next round's samples are loaded
    // from memory while the MFMAs run on this round's, and stored after them
    __shared__ double sA[2][SJ_KC][SJ_TILE + SJ_PAD];
    __shared__ double sB[2][SJ_KC][SJ_TILE + SJ_PAD];
    const int L = blockIdx.x, xcd = L & 7, slot = L >> 3;
    const int rt = (slot / (col_tiles * ks)) * 8 + xcd, rem = slot % (col_tiles * ks);
    const int ct = rem % col_tiles, half = rem / col_tiles;
    if (rt >= row_tiles) return;
    // this workgroup's samples [kbeg, kend): whole rounds, the last split ragged
    const int64_t mk = ((m + ks - 1) / ks + SJ_KC - 1) / SJ_KC * SJ_KC;
    const int64_t kbeg = half * mk, kend = kbeg + mk < m ? kbeg + mk : m;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int64_t i0 = (int64_t)rt * SJ_TILE;   // rows of S_J (variables)
    const int c0 = ct * SJ_TILE;                // block columns
    // loader mapping: 16 rows x 64 columns, 4 consecutive doubles per thread
    const int lr = tid >> 4;          // 0..15
    const int lc = (tid & 15) * 4;    // 0..60
    double4_t acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb) acc[a][bb] = (double4_t){0.0, 0.0, 0.0, 0.0};
    // The next round's loads go out before this round's MFMAs; entries past
    // the matrix read element 0 and are zeroed only when staged, since a
    // select next to the load would wait for it there.
    double ra[4], rb[4];
    auto load = [&](int64_t r0) {
        const int64_t r = r0 + lr;
        const bool rok = r < kend;
        const double* xrow = X + (rok ? r : 0) * n;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int64_t ia = i0 + lc + q;
            const int cb = c0 + lc + q;
            ra[q] = xrow[rok && ia < n ? ia : 0];
            rb[q] = xrow[rok && cb < b ? j0 + cb : 0];
        }
    };
    auto stage = [&](int buf, int64_t r0) {
        const bool rok = r0 + lr < kend;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            sA[buf][lr][lc + q] = rok && i0 + lc + q < n ? ra[q] : 0.0;
            sB[buf][lr][lc + q] = rok && c0 + lc + q < b ? rb[q] : 0.0;
        }
    };
    load(kbeg);
    stage(0, kbeg);
    __syncthreads();
    int buf = 0;
    for (int64_t r0 = kbeg; r0 < kend; r0 += SJ_KC) {
        const bool more = r0 + SJ_KC < kend;
        if (more) load(r0 + SJ_KC);
#pragma unroll
        for (int kk = 0; kk < SJ_KC; kk += 4) {
            const int kr = kk + (lane >> 4);
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = sA[buf][kr][wr * 32 + a * 16 + (lane & 15)];
#pragma unroll
            for (int bb = 0; bb < 2; ++bb) bv[bb] = sB[buf][kr][wc * 32 + bb * 16 + (lane & 15)];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int bb = 0; bb < 2; ++bb)
                    acc[a][bb] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[a], bv[bb], acc[a][bb], 0, 0, 0);
        }
        if (more) stage(buf ^ 1, r0 + SJ_KC);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t i = i0 + wr * 32 + a * 16 + (lane >> 4) + 4 * v;
                const int c = c0 + wc * 32 + bb * 16 + (lane & 15);
                if (i < n && c < b) {
                    if (ks == 1) out[i * b + c] = acc[a][bb][v] * invm;
                    else unsafeAtomicAdd(out + i * b + c, acc[a][bb][v] * invm);
                }
            }
}

// Reduced-precision S_J (the mixed-precision path): the same 64 x 64 tiles,
// float accumulation on MFMA, the result scaled and widened to float64.
//   float X:    v_mfma_f32_16x16x4f32, operands A[l%16][l/16], B[l/16][l%16]
//   bfloat16 X: v_mfma_f32_16x16x16bf16_1k, A[l%16][4(l/16)+q], B[4(l/16)+q][l%16]
// both with the result in D[4(l/16)+v][l%16] (checked with a lane-layout probe).
typedef float float4_t __attribute__((ext_vector_type(4)));
typedef short short4_t __attribute__((ext_vector_type(4)));

constexpr int SJR_KC = 32;    // samples staged per LDS round
constexpr int SJR_PAD = 4;
constexpr int SJR_TPAD = 4;   // bfloat16 staging: [column][sample] rows of SJR_KC + 4 (8-byte aligned)

// Tiles, XCD order, sample split (ks = 1 or 2, atomically added) and double
// buffering as in k_sj_gemm_f64. bfloat16 samples are staged transposed,
// [column][sample], so the four consecutive samples a lane supplies to the
// MFMA are one 8-byte LDS read; float samples [sample][column].
template <bool BF16>
__global__ __launch_bounds__(256) void k_sj_gemm_low(const void* __restrict__ Xv, int64_t n,
                                                     int64_t m, int64_t j0, int b,
                                                     double* __restrict__ out, double invm,
                                                     int row_tiles, int col_tiles, int ks) {
    typedef typename std::conditional<BF16, unsigned short, float>::type E;
    const E* __restrict__ X = (const E*)Xv;
    constexpr int RS = BF16 ? SJR_KC + SJR_TPAD : SJ_TILE + SJR_PAD;   // LDS row stride
    constexpr int NR = BF16 ? SJ_TILE : SJR_KC;                         // LDS rows
    __shared__ __attribute__((aligned(16))) E sA[2][NR * RS];
    __shared__ __attribute__((aligned(16))) E sB[2][NR * RS];
    auto at = [](int k, int col) { return BF16 ? col * RS + k : k * RS + col; };
    const int L = blockIdx.x, xcd = L & 7, slot = L >> 3;
    const int rt = (slot / (col_tiles * ks)) * 8 + xcd, rem = slot % (col_tiles * ks);
    const int ct = rem % col_tiles, half = rem / col_tiles;
    if (rt >= row_tiles) return;
    const int64_t mk = ((m + ks - 1) / ks + SJR_KC - 1) / SJR_KC * SJR_KC;
    const int64_t kbeg = half * mk, kend = kbeg + mk < m ? kbeg + mk : m;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = tid >> 6;
    const int wr = wave >> 1, wc = wave & 1;
    const int64_t i0 = (int64_t)rt * SJ_TILE;
    const int c0 = ct * SJ_TILE;
    // loader: 32 samples x 64 columns, 8 consecutive columns per thread
    const int lr = tid >> 3;          // 0..31
    const int lc = (tid & 7) * 8;     // 0..56
    float4_t acc[2][2];
    for (int a = 0; a < 2; ++a)
        for (int bb = 0; bb < 2; ++bb) acc[a][bb] = (float4_t){0.f, 0.f, 0.f, 0.f};
    E ra[8], rb[8];
    auto load = [&](int64_t r0) {   // raw values; entries past the matrix read element 0
        const int64_t r = r0 + lr;
        const bool rok = r < kend;
        const E* xrow = X + (rok ? r : 0) * n;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const int64_t ia = i0 + lc + q;
            const int cb = c0 + lc + q;
            ra[q] = xrow[rok && ia < n ? ia : 0];
            rb[q] = xrow[rok && cb < b ? j0 + cb : 0];
        }
    };
    auto stage = [&](int buf, int64_t r0) {   // masked here, after the MFMAs
        const bool rok = r0 + lr < kend;
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            sA[buf][at(lr, lc + q)] = rok && i0 + lc + q < n ? ra[q] : (E)0;
            sB[buf][at(lr, lc + q)] = rok && c0 + lc + q < b ? rb[q] : (E)0;
        }
    };
    load(kbeg);
    stage(0, kbeg);
    __syncthreads();
    int buf = 0;
    for (int64_t r0 = kbeg; r0 < kend; r0 += SJR_KC) {
        const bool more = r0 + SJR_KC < kend;
        if (more) load(r0 + SJR_KC);
        if constexpr (BF16) {
#pragma unroll
            for (int kk = 0; kk < SJR_KC; kk += 16) {
                const int kr = kk + 4 * (lane >> 4);
                short4_t av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; ++a)
                    av[a] = *(const short4_t*)&sA[buf][at(kr, wr * 32 + a * 16 + (lane & 15))];
#pragma unroll
                for (int bb = 0; bb < 2; ++bb)
                    bv[bb] = *(const short4_t*)&sB[buf][at(kr, wc * 32 + bb * 16 + (lane & 15))];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int bb = 0; bb < 2; ++bb)
                        acc[a][bb] = __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(av[a], bv[bb],
                                                                              acc[a][bb], 0, 0, 0);
            }
        } else {
#pragma unroll
            for (int kk = 0; kk < SJR_KC; kk += 4) {
                const int kr = kk + (lane >> 4);
                float av[2], bv[2];
#pragma unroll
                for (int a = 0; a < 2; ++a) av[a] = sA[buf][at(kr, wr * 32 + a * 16 + (lane & 15))];
#pragma unroll
                for (int bb = 0; bb < 2; ++bb) bv[bb] = sB[buf][at(kr, wc * 32 + bb * 16 + (lane & 15))];
#pragma unroll
                for (int a = 0; a < 2; ++a)
#pragma unroll
                    for (int bb = 0; bb < 2; ++bb)
                        acc[a][bb] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[a], bv[bb], acc[a][bb],
                                                                          0, 0, 0);
            }
        }
        if (more) stage(buf ^ 1, r0 + SJR_KC);
        __syncthreads();
        buf ^= 1;
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int bb = 0; bb < 2; ++bb)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t i = i0 + wr * 32 + a * 16 + 4 * (lane >> 4) + v;
                const int c = c0 + wc * 32 + bb * 16 + (lane & 15);
                if (i < n && c < b) {
                    const double val = (double)acc[a][bb][v] * invm;
                    if (ks == 1) out[i * b + c] = val;
                    else unsafeAtomicAdd(out + i * b + c, val);
                }
            }
}

// float64 -> float (round to nearest) and -> bfloat16 (round to nearest even)
__global__ void k_narrow(const double* __restrict__ X, int64_t count, float* __restrict__ xf,
                         unsigned short* __restrict__ xb) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= count) return;
    const float f = (float)X[t];
    if (xf) xf[t] = f;
    if (xb) {
        unsigned u = __float_as_uint(f);
        if ((u & 0x7f800000u) == 0x7f800000u) {
            xb[t] = (unsigned short)((u >> 16) | ((u & 0xffffu) ? 0x40u : 0u));   // inf / nan
        } else {
            u += 0x7fffu + ((u >> 16) & 1u);
            xb[t] = (unsigned short)(u >> 16);
        }
    }
}

__global__ __launch_bounds__(256) void k_transpose(const double* __restrict__ X, int64_t m, int64_t n,
                                                   double* __restrict__ Xt) {
    __shared__ double tile[32][33];
    const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;   // 32 x 8
    const int64_t c0 = (int64_t)blockIdx.x * 32;   // column of X (variable)
    const int64_t r0 = (int64_t)blockIdx.y * 32;   // row of X (sample)
    for (int k = ty; k < 32; k += 8) {
        const int64_t r = r0 + k, c = c0 + tx;
        tile[k][tx] = (r < m && c < n) ? X[r * n + c] : 0.0;
    }
    __syncthreads();
    for (int k = ty; k < 32; k += 8) {
        const int64_t c = c0 + k, r = r0 + tx;
        if (c < n && r < m) Xt[c * m + r] = tile[tx][k];
    }
}

__device__ inline double wave_sum(double v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

__global__ __launch_bounds__(256) void k_diag_s(const double* __restrict__ Xt, int64_t n, int64_t m,
                                                double* __restrict__ d, double invm) {
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= n) return;
    const double* x = Xt + i * m;
    double s = 0.0;
    for (int64_t r = lane; r < m; r += 64) s += x[r] * x[r];
    s = wave_sum(s);
    if (lane == 0) d[i] = s * invm;
}

__global__ __launch_bounds__(256) void k_sddmm(const double* __restrict__ Xt, int64_t m,
                                               const int32_t* __restrict__ rows,
                                               const int32_t* __restrict__ cols, int64_t count,
                                               double* __restrict__ out, double invm) {
    const int lane = threadIdx.x & 63;
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (t >= count) return;
    const double* x = Xt + (int64_t)rows[t] * m;
    const double* y = Xt + (int64_t)cols[t] * m;
    double s = 0.0;
    for (int64_t r = lane; r < m; r += 64) s += x[r] * y[r];
    s = wave_sum(s);
    if (lane == 0) out[t] = s * invm;
}

}  // namespace

void launch_sj_gemm_f64(const double* X, int64_t n, int64_t m, int64_t j0, int b, double* out,
                        hipStream_t s) {
    const int row_tiles = (int)((n + SJ_TILE - 1) / SJ_TILE);
    const int col_tiles = (b + SJ_TILE - 1) / SJ_TILE;
    // the samples split in two when there are enough of them to pay for the fill
    const int ks = m >= 256 ? 2 : 1;
    const unsigned grid = (unsigned)(8 * ((row_tiles + 7) / 8) * col_tiles * ks);
    if (ks > 1) SIC_HIP(hipMemsetAsync(out, 0, sizeof(double) * n * b, s));
    prof_begin(KK_SJ, s);
    hipLaunchKernelGGL(k_sj_gemm_f64, dim3(grid), dim3(256), 0, s, X, n, m, j0, b, out,
                       1.0 / (double)m, row_tiles, col_tiles, ks);
    SIC_CHECK_LAUNCH();
    // algorithmic: X read once (m x n) and S_J written once; 2 n b m flops
    prof_end(KK_SJ, s, 8.0 * ((double)m * n + (double)n * b), 2.0 * (double)n * b * m);
}

void launch_sj_gemm_low(const void* X, bool bf16, int64_t n, int64_t m, int64_t j0, int b,
                        double* out, hipStream_t s) {
    const int row_tiles = (int)((n + SJ_TILE - 1) / SJ_TILE);
    const int col_tiles = (b + SJ_TILE - 1) / SJ_TILE;
    const int ks = m >= 256 ? 2 : 1;
    const unsigned grid = (unsigned)(8 * ((row_tiles + 7) / 8) * col_tiles * ks);
    if (ks > 1) SIC_HIP(hipMemsetAsync(out, 0, sizeof(double) * n * b, s));
    const double esz = bf16 ? 2.0 : 4.0;
    prof_begin(bf16 ? KK_SJ_BF16 : KK_SJ_F32, s);
    if (bf16)
        hipLaunchKernelGGL(k_sj_gemm_low<true>, dim3(grid), dim3(256), 0, s, X, n, m, j0, b, out,
                           1.0 / (double)m, row_tiles, col_tiles, ks);
    else
        hipLaunchKernelGGL(k_sj_gemm_low<false>, dim3(grid), dim3(256), 0, s, X, n, m, j0, b, out,
                           1.0 / (double)m, row_tiles, col_tiles, ks);
    SIC_CHECK_LAUNCH();
    prof_end(bf16 ? KK_SJ_BF16 : KK_SJ_F32, s, esz * (double)m * n + 8.0 * (double)n * b,
             2.0 * (double)n * b * m);
}

void launch_narrow(const double* X, int64_t count, float* xf, uint16_t* xb, hipStream_t s) {
    hipLaunchKernelGGL(k_narrow, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, X, count,
                       xf, (unsigned short*)xb);
    SIC_CHECK_LAUNCH();
}

void launch_transpose(const double* X, int64_t m, int64_t n, double* Xt, hipStream_t s) {
    dim3 grid((unsigned)((n + 31) / 32), (unsigned)((m + 31) / 32));
    hipLaunchKernelGGL(k_transpose, grid, dim3(256), 0, s, X, m, n, Xt);
    SIC_CHECK_LAUNCH();
}

void launch_diag_s(const double* Xt, int64_t n, int64_t m, double* d, hipStream_t s) {
    hipLaunchKernelGGL(k_diag_s, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s, Xt, n, m, d,
                       1.0 / (double)m);
    SIC_CHECK_LAUNCH();
}

void launch_sddmm(const double* Xt, int64_t m, const int32_t* rows, const int32_t* cols,
                  int64_t count, double* out, hipStream_t s) {
    if (count <= 0) return;
    prof_begin(KK_SDDMM, s);
    hipLaunchKernelGGL(k_sddmm, dim3((unsigned)((count + 3) / 4)), dim3(256), 0, s, Xt, m, rows,
                       cols, count, out, 1.0 / (double)m);
    SIC_CHECK_LAUNCH();
    prof_end(KK_SDDMM, s, 16.0 * (double)m * count + 16.0 * count, 2.0 * (double)m * count);
}

}  // namespace sic
