// Device kernels of the top-r eigensolver (the eigenpairs U1, L1 that the
// hybrid method takes as input, Section 4.1): Chebyshev-filtered subspace
// iteration in double precision on a block X of m vectors, stored item-major
// (N x m, row i = item i's m entries), so one sparse product gathers whole
// contiguous rows as in the solver's SpMM.
#include "hd_device.h"
#include "hd_kernels.h"

namespace hd {

// splitmix64 (Steele, Lea, Flood 2014): a counter-based 64-bit mixer.
__device__ __forceinline__ uint64_t splitmix64(uint64_t x) {
    x += 0x9E3779B97F4A7C15ull;
    x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
    x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
    return x ^ (x >> 31);
}

// X[i][j] = a standard normal draw from (seed, i*m + j): two uniforms from
// two splitmix64 values, Box-Muller.
__global__ __launch_bounds__(kBlock) void k_eig_rand(int64_t N, int m, uint64_t seed, double *X) {
    const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (size_t)N * m) return;
    const uint64_t a = splitmix64(seed ^ splitmix64(2 * idx));
    const uint64_t b = splitmix64(seed ^ splitmix64(2 * idx + 1));
    const double u1 = ((double)(a >> 11) + 1.0) * (1.0 / 9007199254740993.0);  // (0, 1]
    const double u2 = (double)(b >> 11) * (1.0 / 9007199254740992.0);          // [0, 1)
    X[idx] = sqrt(-2.0 * log(u1)) * cos(6.283185307179586 * u2);
}

hipError_t launch_eig_rand(int64_t N, int m, uint64_t seed, double *X, hipStream_t s) {
    const size_t tot = (size_t)N * m;
    k_eig_rand<<<(unsigned)((tot + kBlock - 1) / kBlock), kBlock, 0, s>>>(N, m, seed, X);
    return hipGetLastError();
}

// Out = a (S Y1) + b Y1 + c Y0 (Y0 may be null) for the N x m item-major
// blocks: one wave per row and 64 columns (grid.y), m a multiple of 64; the
// row's (column, value) pairs are read 64 at a time and broadcast.
__global__ __launch_bounds__(kBlock) void k_eig_cheb(int64_t N, const int64_t *__restrict__ rowptr,
                                                     const int32_t *__restrict__ col,
                                                     const float *__restrict__ val, int m,
                                                     const double *__restrict__ Y1,
                                                     const double *__restrict__ Y0, double *__restrict__ Out,
                                                     double a, double b, double c) {
    const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
    if (i >= N) return;
    const int lane = threadIdx.x % kWave;
    const int j = blockIdx.y * kWave + lane;
    const int64_t beg = rowptr[i], end = rowptr[i + 1];
    double acc = 0.0;
    for (int64_t base = beg; base < end; base += kWave) {
        const int cnt = end - base < kWave ? (int)(end - base) : kWave;
        int ci = 0;
        float cv = 0.f;
        if (lane < cnt) {
            ci = col[base + lane];
            cv = val[base + lane];
        }
        int t = 0;
        for (; t + 4 <= cnt; t += 4) {
            double pv[4], vv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                vv[u] = (double)bcast_f(cv, t + u);
                pv[u] = Y1[(size_t)bcast_i(ci, t + u) * m + j];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc += vv[u] * pv[u];
        }
        for (; t < cnt; ++t) acc += (double)bcast_f(cv, t) * Y1[(size_t)bcast_i(ci, t) * m + j];
    }
    const size_t o = (size_t)i * m + j;
    double v = a * acc + b * Y1[o];
    if (Y0) v += c * Y0[o];
    Out[o] = v;
}

hipError_t launch_eig_cheb(int64_t N, const int64_t *rowptr, const int32_t *col, const float *val, int m,
                           const double *Y1, const double *Y0, double *Out, double a, double b, double c,
                           hipStream_t s) {
    if (m % kWave != 0) return hipErrorInvalidValue;
    k_eig_cheb<<<dim3((unsigned)((N + 3) / 4), (unsigned)(m / kWave)), kBlock, 0, s>>>(N, rowptr, col, val, m, Y1,
                                                                                     Y0, Out, a, b, c);
    return hipGetLastError();
}

// part[blk][j] = sum over the block's rows of (SX[i][j] - w[j] X[i][j])^2;
// a block of 256 threads covers 256 columns (grid.y) of rb rows.
__global__ __launch_bounds__(kBlock) void k_eig_resid(int64_t N, int m, const double *__restrict__ SX,
                                                      const double *__restrict__ X, const double *__restrict__ w,
                                                      int64_t rb, double *__restrict__ part) {
    const int j = blockIdx.y * kBlock + threadIdx.x;
    if (j >= m) return;
    const int64_t r0 = (int64_t)blockIdx.x * rb, r1 = r0 + rb < N ? r0 + rb : N;
    const double wj = w[j];
    double acc = 0.0;
    for (int64_t i = r0; i < r1; ++i) {
        const size_t o = (size_t)i * m + j;
        const double d = SX[o] - wj * X[o];
        acc += d * d;
    }
    part[(size_t)blockIdx.x * m + j] = acc;
}

hipError_t launch_eig_resid(int64_t N, int m, const double *SX, const double *X, const double *w, int64_t rb,
                            int nblk, double *part, hipStream_t s) {
    k_eig_resid<<<dim3((unsigned)nblk, (unsigned)((m + kBlock - 1) / kBlock)), kBlock, 0, s>>>(N, m, SX, X, w, rb,
                                                                                            part);
    return hipGetLastError();
}

// U[i][k] = (float) X[i][k] for k < r (X item-major N x m).
__global__ __launch_bounds__(kBlock) void k_eig_extract(int64_t N, int m, int r, const double *__restrict__ X,
                                                        float *__restrict__ U) {
    const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (size_t)N * r) return;
    const size_t i = idx / r, k = idx % r;
    U[idx] = (float)X[i * m + k];
}

hipError_t launch_eig_extract(int64_t N, int m, int r, const double *X, float *U, hipStream_t s) {
    const size_t tot = (size_t)N * r;
    k_eig_extract<<<(unsigned)((tot + kBlock - 1) / kBlock), kBlock, 0, s>>>(N, m, r, X, U);
    return hipGetLastError();
}

}  // namespace hd
