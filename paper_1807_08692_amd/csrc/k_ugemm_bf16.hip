// BF16 storage form of the eigenvector products (the precision form of the
// low-rank parts of Section 4.2, eqs. (h-spectral) and (box)).
//
// U1 is stored in bfloat16 twice: item-major (N x rp, for U C) and
// component-major (rp x N, for U^T P), so that every MFMA operand a lane
// needs - eight consecutive K elements - is one 16-byte load. The other
// operand (P, or the small coefficient matrix C) stays fp32 in memory and is
// split into hi + lo bfloat16 parts (hi = RNE(v), lo = RNE(v - hi)); each
// product is done twice (hi and lo) into fp32 accumulators, so the only
// approximation beyond fp32 is the bfloat16 storage of U1 itself.
//
// MFMA v_mfma_f32_16x16x32_bf16 operand layout (lane l of 64):
//   A (16 x 32): row l % 16, k = 8*(l/16) .. +7;  B (32 x 16): col l % 16,
//   k = 8*(l/16) .. +7;  C (16 x 16, 4 values): row 4*(l/16) + v, col l % 16.
#include "hd_device.h"
#include "hd_kernels.h"

namespace hd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mfma16bf(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// fp32 -> bf16 bits, round to nearest even (finite inputs).
__device__ __forceinline__ unsigned short bf16_rne(float x) {
    const uint32_t u = __float_as_uint(x);
    return (unsigned short)((u + 0x7fffu + ((u >> 16) & 1u)) >> 16);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) {
    return __uint_as_float((uint32_t)h << 16);
}
// Split eight fp32 values into hi and lo bfloat16 vectors.
__device__ __forceinline__ void split8(const float *v, bf16x8 &hi, bf16x8 &lo) {
    u16x8 h, l;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        const unsigned short hb = bf16_rne(v[q]);
        h[q] = hb;
        l[q] = bf16_rne(v[q] - bf16_to_f(hb));
    }
    hi = __builtin_bit_cast(bf16x8, h);
    lo = __builtin_bit_cast(bf16x8, l);
}
__device__ __forceinline__ bf16x8 load8(const unsigned short *p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(p));
}

// ---------------------------------------------------------------------------
// C^T split: from an fp32 rk x ldb matrix C write CT_hi, CT_lo (ldb x rk
// bfloat16, transposed) for use as the B operand of u_c / combine.
__global__ __launch_bounds__(kBlock) void k_split_t(const float *__restrict__ C, int rk, int ldb,
                                                    unsigned short *__restrict__ CT_hi,
                                                    unsigned short *__restrict__ CT_lo,
                                                    IterGuard ig) {
    if (ig.nact && all_stopped(ig.nact, ig.ntile)) return;
    const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (size_t)rk * ldb) return;
    const int b = (int)(idx / rk), k = (int)(idx % rk);
    const float v = C[(size_t)k * ldb + b];
    const unsigned short h = bf16_rne(v);
    CT_hi[idx] = h;
    CT_lo[idx] = bf16_rne(v - bf16_to_f(h));
}

hipError_t launch_split_t(const float *C, int rk, int ldb, unsigned short *CT_hi,
                          unsigned short *CT_lo, IterGuard g, hipStream_t s) {
    const size_t tot = (size_t)rk * ldb;
    if (tot == 0) return hipSuccess;
    k_split_t<<<(unsigned)((tot + kBlock - 1) / kBlock), kBlock, 0, s>>>(C, rk, ldb, CT_hi, CT_lo, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cpart[c] = U[chunk c]^T P[chunk c] with U component-major bf16 (UT, rp rows
// of stride ldut >= N, a multiple of 64 so that every 8-row run is 16-byte
// aligned).
// M = k (16 per tile), N = b (16), K = rows (32 per MFMA). Wave w owns k
// rows [32w, 32w+32) of the block's 128 (two m-tiles) and the block's 64
// columns (four n-tiles). Per 32-row step the block loads the P tile
// (32 rows x 64 columns, fp32, coalesced), splits it into hi/lo bfloat16 and
// stores it transposed in LDS, so each wave reads its B fragments as 16-byte
// LDS loads; the A fragments come straight from UT. The next step's P tile
// and A fragments are fetched into registers while the current step runs.
__global__ __launch_bounds__(kBlock) void k_ut_p_bf16(int64_t N, const unsigned short *__restrict__ UT,
                                                      int64_t ldut, int rk,
                                                      const float *__restrict__ P, int ldb,
                                                      int64_t rc, float *__restrict__ Cpart,
                                                      IterGuard ig) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    __shared__ __attribute__((aligned(16))) unsigned short Ph[64][40];
    __shared__ __attribute__((aligned(16))) unsigned short Pl[64][40];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    // grid: x = 64-column group (fastest, so the groups of one row chunk run
    // side by side and read U once from memory), y = k group, z = row chunk
    const int k0 = blockIdx.y * 128 + 32 * w;
    const bool kact = k0 < rk;  // waves past rk still help stage P
    const int b0 = blockIdx.x * 64;
    const int64_t rs = (int64_t)blockIdx.z * rc;
    const int64_t re = rs + rc < N ? rs + rc : N;
    const int g = lane / 16, c16 = lane % 16;
    // P staging: thread t -> row t/8 of the tile, columns 8*(t%8) .. +7
    const int prow = threadIdx.x / 8, pcol = 8 * (threadIdx.x % 8);
    f32x4 acc[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};

    float4 pv[2];
    bf16x8 a[2];
    auto fetch = [&](int64_t i) {
        const int64_t r = i + prow;
        if (r < re) {
            const float4 *src = reinterpret_cast<const float4 *>(P + vec_index(N, ldb, r, b0 + pcol));
            pv[0] = src[0];
            pv[1] = src[1];
        } else {
            pv[0] = pv[1] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
        const int64_t r8 = i + 8 * g;
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            if (!kact) {
                a[m] = __builtin_bit_cast(bf16x8, u16x8{0, 0, 0, 0, 0, 0, 0, 0});
                continue;
            }
            const unsigned short *src = UT + (size_t)(k0 + 16 * m + c16) * ldut + r8;
            if (r8 + 8 <= re) {
                a[m] = load8(src);
            } else {
                u16x8 t;
#pragma unroll
                for (int q = 0; q < 8; ++q) t[q] = (r8 + q < re) ? src[q] : (unsigned short)0;
                a[m] = __builtin_bit_cast(bf16x8, t);
            }
        }
    };
    fetch(rs);
    for (int64_t i = rs; i < re; i += 32) {
        __syncthreads();  // previous step's LDS reads are done
        {
            const float v[8] = {pv[0].x, pv[0].y, pv[0].z, pv[0].w, pv[1].x, pv[1].y, pv[1].z, pv[1].w};
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const unsigned short h = bf16_rne(v[q]);
                Ph[pcol + q][prow] = h;
                Pl[pcol + q][prow] = bf16_rne(v[q] - bf16_to_f(h));
            }
        }
        const bf16x8 a0 = a[0], a1 = a[1];
        __syncthreads();
        if (i + 32 < re) fetch(i + 32);
        if (kact) {
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const bf16x8 hi = load8(&Ph[16 * n + c16][8 * g]);
                const bf16x8 lo = load8(&Pl[16 * n + c16][8 * g]);
                acc[0][n] = mfma16bf(a0, hi, acc[0][n]);
                acc[0][n] = mfma16bf(a0, lo, acc[0][n]);
                acc[1][n] = mfma16bf(a1, hi, acc[1][n]);
                acc[1][n] = mfma16bf(a1, lo, acc[1][n]);
            }
        }
    }
    if (!kact) return;
    float *out = Cpart + (size_t)blockIdx.z * rk * ldb;
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n)
#pragma unroll
            for (int v = 0; v < 4; ++v)
                out[(size_t)(k0 + 16 * m + 4 * g + v) * ldb + b0 + 16 * n + c16] = acc[m][n][v];
}

hipError_t launch_ut_p_bf16(int64_t N, const unsigned short *UT, int64_t ldut, int rk, const float *P,
                            int ldb, float *Cpart, IterGuard g, hipStream_t s) {
    int64_t rc;
    const int nchunk = ut_p_chunks(N, &rc);
    const int kgroups = (rk + 127) / 128;
    k_ut_p_bf16<<<dim3(ldb / 64, kgroups, nchunk), kBlock, 0, s>>>(N, UT, ldut, rk, P, ldb, rc, Cpart, g);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// acc += U[rows i0+32w .. +32] x C[:, c0 .. c0+64) over all rk, with U
// item-major bf16 (N x rp) and C given as split transposed CT_hi/lo (ldb x rk).
// The block's 64 columns of CT (hi and lo) for one 32-wide k chunk are
// staged in LDS and shared by the four waves; the A fragments (U rows) come
// straight from memory. The next chunk is fetched into registers while the
// current one is multiplied.
__device__ __forceinline__ void uc_bf16_tile(int64_t N, const unsigned short *__restrict__ U,
                                             int rp, int rk,
                                             const unsigned short *__restrict__ CT_hi,
                                             const unsigned short *__restrict__ CT_lo,
                                             int64_t i0, int c0, f32x4 (*acc)[4]) {
    __shared__ __attribute__((aligned(16))) unsigned short Ch[64][40];
    __shared__ __attribute__((aligned(16))) unsigned short Cl[64][40];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int g = lane / 16, c16 = lane % 16;
    // CT staging: thread t -> column t/4, k 8*(t%4) .. +7 of the chunk
    const int scol = threadIdx.x / 4, sk = 8 * (threadIdx.x % 4);
    int64_t row[2];
    bool ok[2];
#pragma unroll
    for (int m = 0; m < 2; ++m) {
        row[m] = i0 + 32 * w + 16 * m + c16;
        ok[m] = row[m] < N;
    }
    const bf16x8 zero = __builtin_bit_cast(bf16x8, u16x8{0, 0, 0, 0, 0, 0, 0, 0});
    bf16x8 a[2], sh, sl;
    auto fetch = [&](int k0) {
#pragma unroll
        for (int m = 0; m < 2; ++m) a[m] = ok[m] ? load8(U + (size_t)row[m] * rp + k0 + 8 * g) : zero;
        const size_t o = (size_t)(c0 + scol) * rk + k0 + sk;
        sh = load8(CT_hi + o);
        sl = load8(CT_lo + o);
    };
    if (rk > 0) fetch(0);
    for (int k0 = 0; k0 < rk; k0 += 32) {
        __syncthreads();
        *reinterpret_cast<bf16x8 *>(&Ch[scol][sk]) = sh;
        *reinterpret_cast<bf16x8 *>(&Cl[scol][sk]) = sl;
        const bf16x8 a0 = a[0], a1 = a[1];
        __syncthreads();
        if (k0 + 32 < rk) fetch(k0 + 32);
#pragma unroll
        for (int n = 0; n < 4; ++n) {
            const bf16x8 h = load8(&Ch[16 * n + c16][8 * g]);
            const bf16x8 l = load8(&Cl[16 * n + c16][8 * g]);
            acc[0][n] = mfma16bf(a0, h, acc[0][n]);
            acc[0][n] = mfma16bf(a0, l, acc[0][n]);
            acc[1][n] = mfma16bf(a1, h, acc[1][n]);
            acc[1][n] = mfma16bf(a1, l, acc[1][n]);
        }
    }
}

// Z = P + alpha U Cl: a block covers 128 rows x 64 columns (wave w: 32 rows).
__global__ __launch_bounds__(kBlock) void k_u_c_bf16(int64_t N, const unsigned short *__restrict__ U,
                                                     int rp, int rk,
                                                     const unsigned short *__restrict__ CT_hi,
                                                     const unsigned short *__restrict__ CT_lo,
                                                     int ldb, const float *__restrict__ P,
                                                     float alpha, float *__restrict__ Z,
                                                     IterGuard ig) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int g = lane / 16, c16 = lane % 16;
    // grid: x = 64-column group (fastest: the groups of one row block share
    // their U rows through the caches), y = 128-row block
    const int64_t i0 = (int64_t)blockIdx.y * 128;
    const int c0 = blockIdx.x * 64;
    f32x4 acc[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    uc_bf16_tile(N, U, rp, rk, CT_hi, CT_lo, i0, c0, acc);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t i = i0 + 32 * w + 16 * m + 4 * g + v;
            if (i >= N) continue;
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const size_t o = vec_index(N, ldb, i, c0 + 16 * n + c16);
                Z[o] = P[o] + alpha * acc[m][n][v];
            }
        }
}

hipError_t launch_u_c_bf16(int64_t N, const unsigned short *U, int rp, int rk,
                           const unsigned short *CT_hi, const unsigned short *CT_lo, int ldb,
                           const float *P, double alpha, float *Z, IterGuard g, hipStream_t s) {
    dim3 grid((unsigned)(ldb / 64), (unsigned)((N + 127) / 128));
    k_u_c_bf16<<<grid, kBlock, 0, s>>>(N, U, rp, rk, CT_hi, CT_lo, ldb, P, (float)alpha, Z, g);
    return hipGetLastError();
}

// x[b][i] = (U Cs)[i][b] + X[i][b], transposed through LDS (see k_combine).
__global__ __launch_bounds__(kBlock) void k_combine_bf16(int64_t N, int B,
                                                         const unsigned short *__restrict__ U,
                                                         int rp, int rk,
                                                         const unsigned short *__restrict__ CT_hi,
                                                         const unsigned short *__restrict__ CT_lo,
                                                         int ldb, const float *__restrict__ X,
                                                         float *__restrict__ x, int64_t ldx) {
    __shared__ float T[64][129];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int g = lane / 16, c16 = lane % 16;
    const int64_t i0 = (int64_t)blockIdx.y * 128;  // x: query group (fastest), y: row block
    const int c0 = blockIdx.x * 64;
    f32x4 acc[2][4];
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    uc_bf16_tile(N, U, rp, rk, CT_hi, CT_lo, i0, c0, acc);
#pragma unroll
    for (int m = 0; m < 2; ++m)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int rl = 32 * w + 16 * m + 4 * g + v;
            const int64_t i = i0 + rl;
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                const int bl = 16 * n + c16;
                float val = acc[m][n][v];
                if (i < N) val += X[vec_index(N, ldb, i, c0 + bl)];
                T[bl][rl] = val;
            }
        }
    __syncthreads();
    for (int f = threadIdx.x; f < 64 * 128; f += kBlock) {
        const int bl = f / 128, rl = f % 128;
        const int b = c0 + bl;
        const int64_t i = i0 + rl;
        if (b < B && i < N) x[(size_t)b * ldx + i] = T[bl][rl];
    }
}

hipError_t launch_combine_bf16(int64_t N, int B, const unsigned short *U, int rp, int rk,
                               const unsigned short *CT_hi, const unsigned short *CT_lo, int ldb,
                               const float *X, float *x, int64_t ldx, hipStream_t s) {
    dim3 grid((unsigned)((B + 63) / 64), (unsigned)((N + 127) / 128));
    k_combine_bf16<<<grid, kBlock, 0, s>>>(N, B, U, rp, rk, CT_hi, CT_lo, ldb, X, x, ldx);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Query descriptors split once per batch: Qh / Ql (B x ldv bfloat16, zero
// padded), the hi and lo parts of q.
__global__ __launch_bounds__(kBlock) void k_split_q(int B, int d, int ldv, const float *__restrict__ q,
                                                    unsigned short *__restrict__ Qh,
                                                    unsigned short *__restrict__ Ql) {
    const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (size_t)B * ldv) return;
    const int b = (int)(idx / ldv), t = (int)(idx % ldv);
    const float v = t < d ? q[(size_t)b * d + t] : 0.f;
    const unsigned short h = bf16_rne(v);
    Qh[idx] = h;
    Ql[idx] = bf16_rne(v - bf16_to_f(h));
}

// sim[b][j] = q[b] . V[j] with V stored bfloat16 (N x ldv) and q split hi/lo.
// M = b, N = j, K = t. A block covers 64 queries x 256 items; wave w owns
// items [64w, 64w+64) (four n-tiles) for all 64 queries (four m-tiles, hi
// and lo), so each LDS fragment feeds four or eight MFMAs. Per 32-wide k
// chunk the V tile (256 x 32) and the Q tiles (64 x 32, hi and lo) are staged
// in LDS; the next chunk is fetched into registers meanwhile. blockIdx.x runs
// over the query tiles so that the tiles of one item range run together and
// share V through the caches.
__global__ __launch_bounds__(kBlock) void k_sim_bf16(int64_t N, int B, int ldv,
                                                     const unsigned short *__restrict__ Qh,
                                                     const unsigned short *__restrict__ Ql,
                                                     const unsigned short *__restrict__ V,
                                                     float *__restrict__ sim, int64_t lds) {
    __shared__ __attribute__((aligned(16))) unsigned short Vs[256][40];
    __shared__ __attribute__((aligned(16))) unsigned short Qs[2][64][40];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int g = lane / 16, c16 = lane % 16;
    const int b0 = blockIdx.x * 64;
    const int64_t jb = (int64_t)blockIdx.y * 256;
    f32x4 acc[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16x8 zero = __builtin_bit_cast(bf16x8, u16x8{0, 0, 0, 0, 0, 0, 0, 0});
    // staging: V row jb + t (32 values = 4 x 16 B); Q: thread t -> array t/128,
    // row (t%128)/2, k 16*(t%2) .. +15
    const int64_t jv = jb + threadIdx.x;
    const int qa = threadIdx.x / 128, qr = (threadIdx.x % 128) / 2, qk = 16 * (threadIdx.x % 2);
    const unsigned short *qsrc = (qa == 0 ? Qh : Ql) + (size_t)(b0 + qr) * ldv;
    const bool qok = b0 + qr < B;
    bf16x8 vr[4], qv[2];
    auto fetch = [&](int t0) {
#pragma unroll
        for (int u = 0; u < 4; ++u) vr[u] = jv < N ? load8(V + (size_t)jv * ldv + t0 + 8 * u) : zero;
#pragma unroll
        for (int u = 0; u < 2; ++u) qv[u] = qok ? load8(qsrc + t0 + qk + 8 * u) : zero;
    };
    fetch(0);
    for (int t0 = 0; t0 < ldv; t0 += 32) {
        __syncthreads();
#pragma unroll
        for (int u = 0; u < 4; ++u) *reinterpret_cast<bf16x8 *>(&Vs[threadIdx.x][8 * u]) = vr[u];
#pragma unroll
        for (int u = 0; u < 2; ++u) *reinterpret_cast<bf16x8 *>(&Qs[qa][qr][qk + 8 * u]) = qv[u];
        __syncthreads();
        if (t0 + 32 < ldv) fetch(t0 + 32);
        bf16x8 bv[4];
#pragma unroll
        for (int n = 0; n < 4; ++n) bv[n] = load8(&Vs[64 * w + 16 * n + c16][8 * g]);
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            const bf16x8 h = load8(&Qs[0][16 * m + c16][8 * g]);
            const bf16x8 l = load8(&Qs[1][16 * m + c16][8 * g]);
#pragma unroll
            for (int n = 0; n < 4; ++n) {
                acc[m][n] = mfma16bf(h, bv[n], acc[m][n]);
                acc[m][n] = mfma16bf(l, bv[n], acc[m][n]);
            }
        }
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const int64_t j = jb + 64 * w + 16 * n + c16;
        if (j >= N) continue;
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int b = b0 + 16 * m + 4 * g + v;
                if (b < B) sim[(size_t)b * lds + j] = acc[m][n][v];
            }
    }
}

hipError_t launch_sim_bf16(int64_t N, int B, int d, const float *q, const unsigned short *V,
                           int ldv, unsigned short *qsplit, float *sim, int64_t lds, hipStream_t s) {
    unsigned short *Qh = qsplit, *Ql = qsplit + (size_t)B * ldv;
    const size_t tot = (size_t)B * ldv;
    k_split_q<<<(unsigned)((tot + kBlock - 1) / kBlock), kBlock, 0, s>>>(B, d, ldv, q, Qh, Ql);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)((B + 63) / 64), (unsigned)((N + 255) / 256));
    k_sim_bf16<<<grid, kBlock, 0, s>>>(N, B, ldv, Qh, Ql, V, sim, lds);
    return hipGetLastError();
}

}  // namespace hd
