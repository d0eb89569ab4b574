// Tall-skinny eigenvector products on the MFMA units (gfx950, fp32 MFMA
// 32x32x2): the low-rank part U1 L1 U1^T z of the deflated operator of
// Section 4.2, eq. (box), evaluated right to left, and the spectral term of
// eq. (h-spectral) combined with the temporal term (eq. (hybrid)).
//
//   ut_p    : Cpart[c] = U[rows of chunk c]^T P[rows of chunk c]   (split-K)
//   reduce_c: Cl = L1 .* sum_c Cpart[c]            (fixed order, double)
//   u_c     : Z  = P + alpha * U Cl                (so that (Z - alpha S P) /
//                                                   (1 - alpha) is eq. (box))
//   combine : x[b][i] = (U Cs)[i][b] + X[i][b]     (x = x^s + x^t, query-major)
//
// MFMA v_mfma_f32_32x32x2f32 operand layout (lane l of 64):
//   A (32 x 2): A[l % 32][l / 32];  B (2 x 32): B[l / 32][l % 32];
//   C (32 x 32, 16 values): C[8*(v/4) + 4*(l/32) + v%4][l % 32].
#include "hd_device.h"
#include "hd_kernels.h"

namespace hd {

__device__ __forceinline__ f32x16 mfma32(float a, float b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ int acc_row(int v, int lane) {
    return 8 * (v / 4) + 4 * (lane / 32) + (v % 4);
}

int ut_p_chunks(int64_t N, int64_t *rows_per_chunk) {
    // about 256 chunks: enough blocks to fill the chip, few partials to reduce
    int64_t rc = (N + 255) / 256;
    rc = ((rc + 63) / 64) * 64;
    if (rc < 256) rc = 256;
    *rows_per_chunk = rc;
    return (int)((N + rc - 1) / rc);
}

// A = U^T (k x rows): lane reads U[row0 + l/32][k0 + l%32] - 128 contiguous
// bytes per row, coalesced. B = P (rows x b): P[row0 + l/32][b0 + l%32].
// Each wave owns one 32-wide k tile and NT 32-wide column tiles.
template <int NT>
__global__ __launch_bounds__(kBlock) void k_ut_p(int64_t N, const float *__restrict__ U, int rp,
                                                 int rk, const float *__restrict__ P, int ldb,
                                                 int64_t rc, float *__restrict__ Cpart) {
    const int lane = threadIdx.x % kWave;
    const int w = threadIdx.x / kWave;
    const int k0 = (blockIdx.y * 4 + w) * 32;
    if (k0 >= rk) return;  // no block-level synchronisation below
    const int b0 = blockIdx.z * 32 * NT;
    const int64_t rs = (int64_t)blockIdx.x * rc;
    const int64_t re = rs + rc < N ? rs + rc : N;
    const int hi = lane / 32, lo = lane % 32;
    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
        for (int v = 0; v < 16; ++v) acc[t][v] = 0.f;

    int64_t i = rs;
    for (; i + 8 <= re; i += 8) {
        float a[4], b[4][NT];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t row = i + 2 * u + hi;
            a[u] = U[(size_t)row * rp + k0 + lo];
#pragma unroll
            for (int t = 0; t < NT; ++t) b[u][t] = P[(size_t)row * ldb + b0 + t * 32 + lo];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = mfma32(a[u], b[u][t], acc[t]);
    }
    for (; i < re; i += 2) {
        const int64_t row = i + hi;
        float a = 0.f, b[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) b[t] = 0.f;
        if (row < re) {
            a = U[(size_t)row * rp + k0 + lo];
#pragma unroll
            for (int t = 0; t < NT; ++t) b[t] = P[(size_t)row * ldb + b0 + t * 32 + lo];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mfma32(a, b[t], acc[t]);
    }
    float *out = Cpart + (size_t)blockIdx.x * rk * ldb;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v)
            out[(size_t)(k0 + acc_row(v, lane)) * ldb + b0 + t * 32 + lo] = acc[t][v];
}

hipError_t launch_ut_p(int64_t N, const float *U, int rp, int rk, const float *P, int ldb,
                       float *Cpart, hipStream_t s) {
    int64_t rc;
    int nchunk = ut_p_chunks(N, &rc);
    int kgroups = (rk / 32 + 3) / 4;
    if (ldb == 64) {
        k_ut_p<2><<<dim3(nchunk, kgroups, 1), kBlock, 0, s>>>(N, U, rp, rk, P, ldb, rc, Cpart);
    } else {
        k_ut_p<4><<<dim3(nchunk, kgroups, ldb / 128), kBlock, 0, s>>>(N, U, rp, rk, P, ldb, rc,
                                                                       Cpart);
    }
    return hipGetLastError();
}

// Cl = L1 .* sum over chunks of Cpart. A block reduces 64 consecutive
// entries of the rk x ldb matrix: its four waves take the chunks c = w mod 4
// with two accumulators each, then the four wave sums are added in order.
__global__ __launch_bounds__(kBlock) void k_reduce_c(int nchunk, const float *__restrict__ Cpart,
                                                     int rk, int ldb, const double *lam, int r_use,
                                                     float *__restrict__ Cl) {
    __shared__ double sh[4][kWave];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const size_t tot = (size_t)rk * ldb;
    const size_t idx = (size_t)blockIdx.x * kWave + lane;   // tot is a multiple of 64
    double s0 = 0.0, s1 = 0.0;
    int c = w;
    for (; c + 4 < nchunk; c += 8) {
        s0 += (double)Cpart[(size_t)c * tot + idx];
        s1 += (double)Cpart[(size_t)(c + 4) * tot + idx];
    }
    for (; c < nchunk; c += 4) s0 += (double)Cpart[(size_t)c * tot + idx];
    sh[w][lane] = s0 + s1;
    __syncthreads();
    if (w == 0) {
        const double sum = ((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane];
        const int k = (int)(idx / ldb);
        Cl[idx] = k < r_use ? (float)(lam[k] * sum) : 0.f;
    }
}

hipError_t launch_reduce_c(int nchunk, const float *Cpart, int rk, int ldb, const double *lam,
                           int r_use, float *Cl, hipStream_t s) {
    size_t tot = (size_t)rk * ldb;
    k_reduce_c<<<(unsigned)(tot / kWave), kBlock, 0, s>>>(nchunk, Cpart, rk, ldb, lam, r_use, Cl);
    return hipGetLastError();
}

// Stage U[i0 .. i0+64)[k0 .. k0+32) into LDS (row pitch 33 floats, so the
// column-wise MFMA reads below hit distinct banks). 256 threads, 8 floats each.
__device__ __forceinline__ void stage_u_tile(float (*Us)[33], const float *__restrict__ U, int rp,
                                             int64_t N, int64_t i0, int k0) {
    const int t = threadIdx.x;
    const int row = t / 4, kk = (t % 4) * 8;
    const int64_t gi = i0 + row;
    float4 x = make_float4(0.f, 0.f, 0.f, 0.f), y = x;
    if (gi < N) {
        const float4 *src = reinterpret_cast<const float4 *>(U + (size_t)gi * rp + k0 + kk);
        x = src[0];
        y = src[1];
    }
    Us[row][kk + 0] = x.x;
    Us[row][kk + 1] = x.y;
    Us[row][kk + 2] = x.z;
    Us[row][kk + 3] = x.w;
    Us[row][kk + 4] = y.x;
    Us[row][kk + 5] = y.y;
    Us[row][kk + 6] = y.z;
    Us[row][kk + 7] = y.w;
}

// Z = P + alpha U Cl over a 64-row x (64*NT)-column tile; the four waves
// split it 2 (rows) x 2 (columns). A = U (rows x k) from LDS, B = Cl (k x b)
// straight from global memory (small, cache resident).
template <int NT>
__global__ __launch_bounds__(kBlock) void k_u_c(int64_t N, const float *__restrict__ U, int rp,
                                                int rk, const float *__restrict__ Cl, int ldb,
                                                const float *__restrict__ P, float alpha,
                                                float *__restrict__ Z) {
    __shared__ float Us[64][33];
    const int lane = threadIdx.x % kWave;
    const int w = threadIdx.x / kWave;
    const int hi = lane / 32, lo = lane % 32;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int wr = (w & 1) * 32;
    const int wc = blockIdx.y * 64 * NT + (w >> 1) * 32 * NT;
    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
        for (int v = 0; v < 16; ++v) acc[t][v] = 0.f;
    for (int k0 = 0; k0 < rk; k0 += 32) {
        stage_u_tile(Us, U, rp, N, i0, k0);
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 32; kk += 2) {
            const float a = Us[wr + lo][kk + hi];
            const float *crow = Cl + (size_t)(k0 + kk + hi) * ldb + wc + lo;
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = mfma32(a, crow[t * 32], acc[t]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t i = i0 + wr + acc_row(v, lane);
            if (i < N) {
                const size_t o = (size_t)i * ldb + wc + t * 32 + lo;
                Z[o] = P[o] + alpha * acc[t][v];
            }
        }
}

hipError_t launch_u_c(int64_t N, const float *U, int rp, int rk, const float *Cl, int ldb,
                      const float *P, double alpha, float *Z, hipStream_t s) {
    const unsigned gx = (unsigned)((N + 63) / 64);
    if (ldb == 64) {
        k_u_c<1><<<dim3(gx, 1), kBlock, 0, s>>>(N, U, rp, rk, Cl, ldb, P, (float)alpha, Z);
    } else if (ldb == 128) {
        k_u_c<2><<<dim3(gx, 1), kBlock, 0, s>>>(N, U, rp, rk, Cl, ldb, P, (float)alpha, Z);
    } else {
        k_u_c<4><<<dim3(gx, ldb / 256), kBlock, 0, s>>>(N, U, rp, rk, Cl, ldb, P, (float)alpha, Z);
    }
    return hipGetLastError();
}

// x^T tile: rows of the product are queries b, columns are items i, so each
// store writes 32 consecutive items of one query. A = Cs^T (b x k) from
// global memory; B = U^T (k x i) from the staged U tile. X (node-major) is
// staged through LDS to add the temporal term in the transposed layout.
__global__ __launch_bounds__(kBlock) void k_combine(int64_t N, int B, const float *__restrict__ U,
                                                    int rp, int rk, const float *__restrict__ Cs,
                                                    int ldb, const float *__restrict__ X,
                                                    float *__restrict__ x, int64_t ldx) {
    __shared__ float Us[64][33];
    __shared__ float Xs[64][65];
    const int lane = threadIdx.x % kWave;
    const int w = threadIdx.x / kWave;
    const int hi = lane / 32, lo = lane % 32;
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int bt = blockIdx.y * 64;
    const int wb = (w & 1) * 32;   // query offset of this wave
    const int wi = (w >> 1) * 32;  // item offset of this wave
    // stage X[i0..i0+64)[bt..bt+64)
    for (int t = threadIdx.x; t < 64 * 16; t += kBlock) {
        const int row = t / 16, c4 = (t % 16) * 4;
        const int64_t gi = i0 + row;
        float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
        if (gi < N) v = *reinterpret_cast<const float4 *>(X + (size_t)gi * ldb + bt + c4);
        Xs[row][c4 + 0] = v.x;
        Xs[row][c4 + 1] = v.y;
        Xs[row][c4 + 2] = v.z;
        Xs[row][c4 + 3] = v.w;
    }
    f32x16 acc;
    for (int v = 0; v < 16; ++v) acc[v] = 0.f;
    for (int k0 = 0; k0 < rk; k0 += 32) {
        __syncthreads();
        stage_u_tile(Us, U, rp, N, i0, k0);
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 32; kk += 2) {
            const float a = Cs[(size_t)(k0 + kk + hi) * ldb + bt + wb + lo];
            const float b = Us[wi + lo][kk + hi];
            acc = mfma32(a, b, acc);
        }
    }
    __syncthreads();
    const int64_t i = i0 + wi + lo;
    if (i < N) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int bl = wb + acc_row(v, lane);
            const int b = bt + bl;
            if (b < B) x[(size_t)b * ldx + i] = acc[v] + Xs[wi + lo][bl];
        }
    }
}

hipError_t launch_combine(int64_t N, int B, const float *U, int rp, int rk, const float *Cs,
                          int ldb, const float *X, float *x, int64_t ldx, hipStream_t s) {
    dim3 grid((unsigned)((N + 63) / 64), (unsigned)((B + 63) / 64));
    k_combine<<<grid, kBlock, 0, s>>>(N, B, U, rp, rk, Cs, ldb, X, x, ldx);
    return hipGetLastError();
}

}  // namespace hd
