// Query-database similarities for the observation vector (Section 3: y holds
// the similarities of the query's nearest neighbours in the dataset; Section
// 6.1: (v^T z)_+^3 on unit-norm descriptors, so v^T z is the cosine).
//
//   sim[b][j] = sum_t q[b][t] * V[j][t]
//
// fp32 MFMA (32x32x2). A block computes 64 queries x 256 database items;
// wave w owns items [64w, 64w+64) for all 64 queries (four 32x32
// accumulators), so every LDS operand feeds two MFMAs. Per 32-wide k chunk
// the block stages Q[64][32] and V[256][32] in LDS; the next chunk is fetched
// into registers while the current one is multiplied. V is streamed from
// HBM once per 64-query tile; stores write 32 consecutive items of a query.
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
    __shared__ float Vs[256][33];
    const int t = threadIdx.x;
    const int lane = t % kWave, w = t / kWave;
    const int hi = lane / 32, lo = lane % 32;
    // logical tiles: 64-query tile fastest (the tiles of one item range share
    // V through one XCD's L2), then 256-item range
    const unsigned L = xcd_tile(), nqt = (unsigned)(B + 63) / 64;
    const int64_t j0 = (int64_t)(L / nqt) * 256;
    const int b0 = (int)(L % nqt) * 64;
    f32x16 acc[2][2];
    for (int m = 0; m < 2; ++m)
        for (int n = 0; n < 2; ++n)
            for (int v = 0; v < 16; ++v) acc[m][n][v] = 0.f;

    // register stage: V row t (32 floats), Q row t/4 (8 floats)
    float4 vr[8];
    float qr[8];
    const int64_t jv = j0 + t;
    const int qrow = t / 4, qk = (t % 4) * 8;
    auto fetch = [&](int k0) {
        if (jv < N) {
            const float4 *src = reinterpret_cast<const float4 *>(V + (size_t)jv * ldv + k0);
#pragma unroll
            for (int m = 0; m < 8; ++m) vr[m] = src[m];
        } else {
#pragma unroll
            for (int m = 0; m < 8; ++m) vr[m] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        const int b = b0 + qrow;
#pragma unroll
        for (int u = 0; u < 8; ++u) {
            const int k = k0 + qk + u;
            qr[u] = (b < B && k < d) ? q[(size_t)b * d + k] : 0.f;
        }
    };
    fetch(0);
    for (int k0 = 0; k0 < d; k0 += 32) {
        __syncthreads();
#pragma unroll
        for (int m = 0; m < 8; ++m) {
            Vs[t][4 * m + 0] = vr[m].x;
            Vs[t][4 * m + 1] = vr[m].y;
            Vs[t][4 * m + 2] = vr[m].z;
            Vs[t][4 * m + 3] = vr[m].w;
        }
#pragma unroll
        for (int u = 0; u < 8; ++u) Qs[qrow][qk + u] = qr[u];
        __syncthreads();
        if (k0 + 32 < d) fetch(k0 + 32);
#pragma unroll 4
        for (int kk = 0; kk < 32; kk += 2) {
            const float a0 = Qs[lo][kk + hi], a1 = Qs[32 + lo][kk + hi];
            const float v0 = Vs[64 * w + lo][kk + hi], v1 = Vs[64 * w + 32 + lo][kk + hi];
            acc[0][0] = mfma32s(a0, v0, acc[0][0]);
            acc[0][1] = mfma32s(a0, v1, acc[0][1]);
            acc[1][0] = mfma32s(a1, v0, acc[1][0]);
            acc[1][1] = mfma32s(a1, v1, acc[1][1]);
        }
    }
#pragma unroll
    for (int n = 0; n < 2; ++n) {
        const int64_t j = j0 + 64 * w + 32 * n + lo;
        if (j >= N) continue;
#pragma unroll
        for (int m = 0; m < 2; ++m)
#pragma unroll
            for (int v = 0; v < 16; ++v) {
                const int b = b0 + 32 * m + 8 * (v / 4) + 4 * hi + (v % 4);
                if (b < B) sim[(size_t)b * lds + j] = acc[m][n][v];
            }
    }
}

hipError_t launch_sim(int64_t N, int B, int d, const float *q, const float *V, int ldv, float *sim,
                      int64_t lds, hipStream_t s) {
    const unsigned nblk = (unsigned)((N + 255) / 256) * (unsigned)((B + 63) / 64);
    k_sim<<<nblk, kBlock, 0, s>>>(N, B, d, q, V, ldv, sim, lds);
    return hipGetLastError();
}

}  // namespace hd
