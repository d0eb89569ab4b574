// SHybrid (Section 6.2): the hybrid method with U1 sparsified, its smallest
// entries set to zero (a global magnitude threshold, no renormalisation, as
// the paper describes), so that the eigenvector products of eqs.
// (h-spectral) and (box) become sparse products. U~ (N x r) is stored twice,
// by item (CSR: the components present in item i's row) for U~ C and the
// final combine, and by component (CSC: the items present in column k) for
// U~^T P and U~^T y.
//
// gfx950 mapping, as for the graph product: one wavefront per output row (an
// item for U~ C, a component for U~^T P), the 64 lanes covering 64 query
// columns each, so every gathered row of the dense operand (C: rk x ldb, in
// L2; P: N x ldb) is one coalesced 256-byte piece per wave. Entries are
// consumed in storage order, so sums are deterministic.
#include "hd_device.h"
#include "hd_kernels.h"

namespace hd {

// acc += sum over entries e in [beg, end) of val[e] * X[idx[e]][c], for the
// lane's column c (X row stride ldx). Each wave fetches 64 (index, value)
// pairs at a time and broadcasts them; four gathers are kept in flight.
__device__ __forceinline__ float wave_row_gather(int64_t beg, int64_t end, const int32_t *__restrict__ idx,
                                                 const float *__restrict__ val,
                                                 const float *__restrict__ X, int64_t ldx, int c) {
    const int lane = threadIdx.x % kWave;
    float acc = 0.f;
    for (int64_t base = beg; base < end; base += kWave) {
        const int cnt = end - base < kWave ? (int)(end - base) : kWave;
        int ci = 0;
        float cv = 0.f;
        if (lane < cnt) {
            ci = idx[base + lane];
            cv = val[base + lane];
        }
        int t = 0;
        for (; t + 4 <= cnt; t += 4) {
            float pv[4], vv[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                vv[u] = bcast_f(cv, t + u);
                pv[u] = X[(size_t)bcast_i(ci, t + u) * ldx + c];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) acc += vv[u] * pv[u];
        }
        for (; t < cnt; ++t) acc += bcast_f(cv, t) * X[(size_t)bcast_i(ci, t) * ldx + c];
    }
    return acc;
}

// Cl[k][b] = lambda_k (U~^T P)[k][b] for k < r_use, 0 for r_use <= k < rk.
// Block = one wave = one component k and 64 columns (blockIdx.y).
__global__ __launch_bounds__(kWave) void k_sp_utp(int rk, int r_use, const int64_t *__restrict__ cptr,
                                                  const int32_t *__restrict__ crow,
                                                  const float *__restrict__ cval,
                                                  const float *__restrict__ P, int ldb,
                                                  const double *__restrict__ lam, float *__restrict__ Cl,
                                                  IterGuard ig) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    const int k = blockIdx.x;
    const int c = blockIdx.y * kWave + threadIdx.x;
    float v = 0.f;
    if (k < r_use) v = (float)lam[k] * wave_row_gather(cptr[k], cptr[k + 1], crow, cval, P, ldb, c);
    Cl[(size_t)k * ldb + c] = v;
}

hipError_t launch_sp_utp(int rk, int r_use, const int64_t *cptr, const int32_t *crow, const float *cval,
                         const float *P, int ldb, const double *lam, float *Cl, IterGuard g, hipStream_t s) {
    if (rk == 0) return hipSuccess;
    k_sp_utp<<<dim3((unsigned)rk, (unsigned)(ldb / kWave)), kWave, 0, s>>>(rk, r_use, cptr, crow, cval, P, ldb,
                                                                           lam, Cl, g);
    return hipGetLastError();
}

// Z[i][b] = P[i][b] + alpha (U~ Cl)[i][b]. Block = four waves, one item each.
__global__ __launch_bounds__(kBlock) void k_sp_uc(int64_t N, const int64_t *__restrict__ rptr,
                                                  const int32_t *__restrict__ rcol,
                                                  const float *__restrict__ rval,
                                                  const float *__restrict__ Cl, int ldb,
                                                  const float *__restrict__ P, float alpha,
                                                  float *__restrict__ Z, IterGuard ig) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    const int64_t i = (int64_t)blockIdx.x * 4 + threadIdx.x / kWave;
    if (i >= N) return;
    const int c = blockIdx.y * kWave + threadIdx.x % kWave;
    const float acc = wave_row_gather(rptr[i], rptr[i + 1], rcol, rval, Cl, ldb, c);
    const size_t o = vec_index(N, ldb, i, c);
    Z[o] = P[o] + alpha * acc;
}

hipError_t launch_sp_uc(int64_t N, const int64_t *rptr, const int32_t *rcol, const float *rval,
                        const float *Cl, int ldb, const float *P, double alpha, float *Z, IterGuard g,
                        hipStream_t s) {
    k_sp_uc<<<dim3((unsigned)((N + 3) / 4), (unsigned)(ldb / kWave)), kBlock, 0, s>>>(
        N, rptr, rcol, rval, Cl, ldb, P, (float)alpha, Z, g);
    return hipGetLastError();
}

// Section 4.2, eq. (h-spectral) with U~: c = U~^T y over the k_y items of y.
// Thread (k, b): scans each y item's CSR row for component k (rows are
// sorted by component). Cs = g(lambda) c, Cl = lambda c (the first
// product's coefficients, P0 = y), in double.
__global__ __launch_bounds__(kBlock) void k_sp_gather_proj(int B, int ky, const int32_t *__restrict__ ids,
                                                           const float *__restrict__ vals, int64_t N,
                                                           const int64_t *__restrict__ rptr,
                                                           const int32_t *__restrict__ rcol,
                                                           const float *__restrict__ rval, int rk,
                                                           int r_use, const double *__restrict__ lam,
                                                           double alpha, int ldb, float *__restrict__ Cs,
                                                           float *__restrict__ Cl,
                                                           const int32_t *__restrict__ colmap,
                                                           const double *__restrict__ gv) {
    const int k = blockIdx.x * kBlock + threadIdx.x;
    const int b = blockIdx.y;
    if (k >= rk) return;
    if (colmap && b >= B) return;
    const int col = colmap ? colmap[b] : b;
    double acc = 0.0;
    if (k < r_use && b < B) {
        for (int t = 0; t < ky; ++t) {
            const int id = ids[b * ky + t];
            if (id < 0 || (int64_t)id >= N) continue;
            for (int64_t e = rptr[id]; e < rptr[id + 1]; ++e) {
                const int kk = rcol[e];
                if (kk >= k) {
                    if (kk == k) acc += (double)rval[e] * (double)vals[b * ky + t];
                    break;
                }
            }
        }
    }
    const double lk = k < r_use ? lam[k] : 0.0;
    const double h = (1.0 - alpha) / (1.0 - alpha * lk);
    const double g = gv ? (k < r_use ? gv[k] : 0.0) : h - (1.0 - alpha);
    Cs[(size_t)k * ldb + col] = (float)(g * acc);
    if (Cl) Cl[(size_t)k * ldb + col] = (float)(lk * acc);
}

hipError_t launch_sp_gather_proj(int B, int ky, const int32_t *ids, const float *vals, int64_t N,
                                 const int64_t *rptr, const int32_t *rcol, const float *rval, int rk,
                                 int r_use, const double *lam, double alpha, int ldb, float *Cs, float *Cl,
                                 hipStream_t s, const int32_t *colmap, const double *gv) {
    if (rk == 0) return hipSuccess;
    dim3 grid((unsigned)((rk + kBlock - 1) / kBlock), (unsigned)(colmap ? B : ldb));
    k_sp_gather_proj<<<grid, kBlock, 0, s>>>(B, ky, ids, vals, N, rptr, rcol, rval, rk, r_use, lam, alpha, ldb,
                                             Cs, Cl, colmap, gv);
    return hipGetLastError();
}

// x[b][i] = (U~ Cs)[i][b] + X[i][b] for b < B: a block covers 64 items x 64
// queries (wave w: items 16w .. +15, lane = query); the tile is transposed
// through LDS so each query's 64 items are written as one run.
__global__ __launch_bounds__(kBlock) void k_sp_combine(int64_t N, int B, const int64_t *__restrict__ rptr,
                                                       const int32_t *__restrict__ rcol,
                                                       const float *__restrict__ rval,
                                                       const float *__restrict__ Cs, int ldc,
                                                       const float *__restrict__ X, float *__restrict__ x,
                                                       int64_t ldx) {
    __shared__ float T[64][65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int b0 = blockIdx.y * 64;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    for (int q = 0; q < 16; ++q) {
        const int rl = 16 * w + q;
        const int64_t i = i0 + rl;
        float v = 0.f;
        if (i < N)
            v = wave_row_gather(rptr[i], rptr[i + 1], rcol, rval, Cs, ldc, b0 + lane) +
                X[vec_index(N, ldc, i, b0 + lane)];
        T[lane][rl] = v;
    }
    __syncthreads();
    for (int f = threadIdx.x; f < 64 * 64; f += kBlock) {
        const int bl = f / 64, rl = f % 64;
        const int b = b0 + bl;
        const int64_t i = i0 + rl;
        if (b < B && i < N) x[(size_t)b * ldx + i] = T[bl][rl];
    }
}

hipError_t launch_sp_combine(int64_t N, int B, const int64_t *rptr, const int32_t *rcol, const float *rval,
                             const float *Cs, int ldc, const float *X, float *x, int64_t ldx, hipStream_t s) {
    k_sp_combine<<<dim3((unsigned)((N + 63) / 64), (unsigned)((B + 63) / 64)), kBlock, 0, s>>>(
        N, B, rptr, rcol, rval, Cs, ldc, X, x, ldx);
    return hipGetLastError();
}

}  // namespace hd
