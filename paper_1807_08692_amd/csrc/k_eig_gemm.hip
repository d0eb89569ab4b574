// Dense double-precision products of the top-r eigensolver's N x m blocks
// (the off-line input of Section 4.1; see hd_eig.cpp) on the FP64 matrix
// cores, v_mfma_f64_16x16x4f64:
//   gram   : G = A^T B  (m x m; A, B item-major N x m; the Gram matrix of
//            CholeskyQR and the Rayleigh quotient X^T S X)
//   rotate : Y = X Z    (N x m; Z m x m column-major: a Ritz rotation, or the
//            inverse Cholesky factor of CholeskyQR)
// Both are exact-order double products: every element of G is summed over
// fixed row chunks in a fixed order, then the chunks in order; Y over its
// 32-wide k steps in order.
//
// v_mfma_f64_16x16x4f64 operand layout (lane l of 64):
//   A (16 x 4): A[l % 16][l / 16];  B (4 x 16): B[l / 16][l % 16];
//   D (16 x 16, 4 doubles): D[l / 16 + 4 v][l % 16] (the double-precision
//   accumulator interleaves its rows: one row per register per lane group,
//   unlike the four consecutive rows of the fp32 16 x 16 forms).
#include "hd_device.h"
#include "hd_kernels.h"

namespace hd {

typedef double f64x4 __attribute__((ext_vector_type(4)));

__device__ __forceinline__ f64x4 mfma_f64(double a, double b, f64x4 c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

constexpr int kEgTile = 64;   // output tile (rows x columns) per block
constexpr int kEgK = 32;      // k rows staged per step
constexpr int64_t kEgChunk = 65536;  // rows per partial Gram matrix

int64_t gram_chunks(int64_t N) { return (N + kEgChunk - 1) / kEgChunk; }

// Gpart[c][p][q] = sum over rows k of chunk c of A[k][p] B[k][q], for the
// 64 x 64 tile (p0, q0). Wave w owns the 32 x 32 quarter (w / 2, w % 2) of
// the tile: 2 x 2 MFMA tiles.
__global__ __launch_bounds__(kBlock) void k_gram_tn(int64_t N, int m, const double *__restrict__ A,
                                                    const double *__restrict__ B, double *__restrict__ Gpart) {
    __shared__ double As[kEgK][kEgTile + 1];
    __shared__ double Bs[kEgK][kEgTile + 1];
    const int ntile = m / kEgTile;
    const int tile = blockIdx.x % (ntile * ntile);
    const int64_t chunk = blockIdx.x / (ntile * ntile);
    const int p0 = (tile / ntile) * kEgTile, q0 = (tile % ntile) * kEgTile;
    const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
    const int wp = (w / 2) * 32, wq = (w % 2) * 32;
    const int64_t ks = chunk * kEgChunk;
    const int64_t ke = ks + kEgChunk < N ? ks + kEgChunk : N;
    f64x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int64_t k0 = ks; k0 < ke; k0 += kEgK) {
        // stage 32 rows x 64 columns of A and of B (rows past ke are zero)
        for (int e = t; e < kEgK * kEgTile; e += kBlock) {
            const int r = e / kEgTile, cc = e % kEgTile;
            const int64_t k = k0 + r;
            As[r][cc] = k < ke ? A[(size_t)k * m + p0 + cc] : 0.0;
            Bs[r][cc] = k < ke ? B[(size_t)k * m + q0 + cc] : 0.0;
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kEgK; kk += 4) {
            const int kr = kk + lane / 16;
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = As[kr][wp + 16 * a + lane % 16];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Bs[kr][wq + 16 * b + lane % 16];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = mfma_f64(av[a], bv[b], acc[a][b]);
        }
        __syncthreads();
    }
    double *out = Gpart + (size_t)chunk * m * m;
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int p = p0 + wp + 16 * a + lane / 16 + 4 * v;
                const int q = q0 + wq + 16 * b + lane % 16;
                out[(size_t)p * m + q] = acc[a][b][v];
            }
}

// G = sum of the chunk partials in chunk order.
__global__ __launch_bounds__(kBlock) void k_gram_reduce(int64_t nchunk, size_t mm, const double *__restrict__ Gpart,
                                                        double *__restrict__ G) {
    const size_t e = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (e >= mm) return;
    double s = 0.0;
    for (int64_t c = 0; c < nchunk; ++c) s += Gpart[(size_t)c * mm + e];
    G[e] = s;
}

// Y[i][q] = sum_p X[i][p] Z[p][q], Z column-major (Z[p][q] at Z[q * ldz + p]);
// a block covers 64 rows x 64 columns of Y, wave w the 32 x 32 quarter.
__global__ __launch_bounds__(kBlock) void k_rotate_nn(int64_t N, int m, const double *__restrict__ X,
                                                      const double *__restrict__ Z, int ldz, double *__restrict__ Y) {
    __shared__ double Xs[kEgTile][kEgK + 1];
    __shared__ double Zs[kEgK][kEgTile + 1];
    const int ncol = m / kEgTile;
    const int q0 = (blockIdx.x % ncol) * kEgTile;
    const int64_t i0 = (int64_t)(blockIdx.x / ncol) * kEgTile;
    const int t = threadIdx.x, lane = t % kWave, w = t / kWave;
    const int wi = (w / 2) * 32, wq = (w % 2) * 32;
    f64x4 acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f64x4{0.0, 0.0, 0.0, 0.0};
    for (int p0 = 0; p0 < m; p0 += kEgK) {
        for (int e = t; e < kEgTile * kEgK; e += kBlock) {
            const int r = e / kEgK, cc = e % kEgK;
            const int64_t i = i0 + r;
            Xs[r][cc] = i < N ? X[(size_t)i * m + p0 + cc] : 0.0;
        }
        for (int e = t; e < kEgK * kEgTile; e += kBlock) {
            const int pr = e % kEgK, cq = e / kEgK;
            Zs[pr][cq] = Z[(size_t)(q0 + cq) * ldz + p0 + pr];
        }
        __syncthreads();
#pragma unroll
        for (int kk = 0; kk < kEgK; kk += 4) {
            const int kr = kk + lane / 16;
            double av[2], bv[2];
#pragma unroll
            for (int a = 0; a < 2; ++a) av[a] = Xs[wi + 16 * a + lane % 16][kr];
#pragma unroll
            for (int b = 0; b < 2; ++b) bv[b] = Zs[kr][wq + 16 * b + lane % 16];
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b) acc[a][b] = mfma_f64(av[a], bv[b], acc[a][b]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t i = i0 + wi + 16 * a + lane / 16 + 4 * v;
                const int q = q0 + wq + 16 * b + lane % 16;
                if (i < N) Y[(size_t)i * m + q] = acc[a][b][v];
            }
}

hipError_t launch_gram(int64_t N, int m, const double *A, const double *B, double *Gpart, double *G, hipStream_t s) {
    if (m % kEgTile != 0 || m <= 0 || N <= 0) return hipErrorInvalidValue;
    const int ntile = m / kEgTile;
    const int64_t nchunk = gram_chunks(N);
    const int64_t blocks = (int64_t)ntile * ntile * nchunk;
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    k_gram_tn<<<(unsigned)blocks, kBlock, 0, s>>>(N, m, A, B, Gpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const size_t mm = (size_t)m * m;
    k_gram_reduce<<<(unsigned)((mm + kBlock - 1) / kBlock), kBlock, 0, s>>>(nchunk, mm, Gpart, G);
    return hipGetLastError();
}

hipError_t launch_rotate(int64_t N, int m, const double *X, const double *Z, int ldz, double *Y, hipStream_t s) {
    if (m % kEgTile != 0 || m <= 0 || N <= 0 || ldz < m || X == Y) return hipErrorInvalidValue;
    const int64_t blocks = (int64_t)(m / kEgTile) * ((N + kEgTile - 1) / kEgTile);
    if (blocks > 0x7fffffff) return hipErrorInvalidValue;
    k_rotate_nn<<<(unsigned)blocks, kBlock, 0, s>>>(N, m, X, Z, ldz, Y);
    return hipGetLastError();
}

}  // namespace hd
