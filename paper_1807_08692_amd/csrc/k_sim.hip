// Query-database similarities for the observation vector (Section 3: y holds
// the similarities of the query's nearest neighbours in the dataset; Section
// 6.1: (v^T z)_+^3 on unit-norm descriptors, so v^T z is the cosine).
//
//   sim[b][j] = sum_t q[b][t] * V[j][t]
//
// fp32 MFMA (32x32x2) with both operands staged through LDS. A block computes
// 64 queries x 128 database items; wave w owns items [32w, 32w+32) for both
// 32-query halves, so a store writes 32 consecutive items of one query.
// V is streamed from HBM once per 64-query tile.
#include "hd_device.h"
#include "hd_kernels.h"

namespace hd {

__device__ __forceinline__ f32x16 mfma32s(float a, float b, f32x16 c) {
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}

__global__ __launch_bounds__(kBlock) void k_sim(int64_t N, int B, int d,
                                                const float *__restrict__ q,
                                                const float *__restrict__ V, int ldv,
                                                float *__restrict__ sim, int64_t lds) {
    __shared__ float Qs[64][33];
    __shared__ float Vs[128][33];
    const int t = threadIdx.x;
    const int lane = t % kWave, w = t / kWave;
    const int hi = lane / 32, lo = lane % 32;
    const int64_t j0 = (int64_t)blockIdx.x * 128;
    const int b0 = blockIdx.y * 64;
    f32x16 acc0, acc1;
    for (int v = 0; v < 16; ++v) {
        acc0[v] = 0.f;
        acc1[v] = 0.f;
    }
    for (int k0 = 0; k0 < d; k0 += 32) {
        {   // Q tile: 64 rows x 32, thread t -> row t/4, 8 consecutive columns
            const int row = t / 4, kk = (t % 4) * 8;
            const int b = b0 + row;
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = k0 + kk + u;
                Qs[row][kk + u] = (b < B && k < d) ? q[(size_t)b * d + k] : 0.f;
            }
        }
        {   // V tile: 128 rows x 32 (V rows padded to ldv, a multiple of 32)
            const int row = t / 2, kk = (t % 2) * 16;
            const int64_t j = j0 + row;
            float4 x[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) x[u] = make_float4(0.f, 0.f, 0.f, 0.f);
            if (j < N) {
                const float4 *src = reinterpret_cast<const float4 *>(V + (size_t)j * ldv + k0 + kk);
#pragma unroll
                for (int u = 0; u < 4; ++u) x[u] = src[u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                Vs[row][kk + 4 * u + 0] = x[u].x;
                Vs[row][kk + 4 * u + 1] = x[u].y;
                Vs[row][kk + 4 * u + 2] = x[u].z;
                Vs[row][kk + 4 * u + 3] = x[u].w;
            }
        }
        __syncthreads();
#pragma unroll 4
        for (int kk = 0; kk < 32; kk += 2) {
            const float bv = Vs[w * 32 + lo][kk + hi];
            acc0 = mfma32s(Qs[lo][kk + hi], bv, acc0);
            acc1 = mfma32s(Qs[32 + lo][kk + hi], bv, acc1);
        }
        __syncthreads();
    }
    const int64_t j = j0 + w * 32 + lo;
    if (j < N) {
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int m = 8 * (v / 4) + 4 * hi + (v % 4);
            if (b0 + m < B) sim[(size_t)(b0 + m) * lds + j] = acc0[v];
            if (b0 + 32 + m < B) sim[(size_t)(b0 + 32 + m) * lds + j] = acc1[v];
        }
    }
}

hipError_t launch_sim(int64_t N, int B, int d, const float *q, const float *V, int ldv, float *sim,
                      int64_t lds, hipStream_t s) {
    dim3 grid((unsigned)((N + 127) / 128), (unsigned)((B + 63) / 64));
    k_sim<<<grid, kBlock, 0, s>>>(N, B, d, q, V, ldv, sim, lds);
    return hipGetLastError();
}

}  // namespace hd
