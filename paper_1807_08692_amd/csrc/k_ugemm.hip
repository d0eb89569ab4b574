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
// Each wave owns one 32-wide k tile and NT 32-wide column tiles. The row loop
// is software pipelined: the operands of the next 16 rows are loaded while
// the MFMAs of the current 16 rows run, so ~24 loads per wave are in flight.
template <int NT>
__global__ __launch_bounds__(kBlock) void k_ut_p(int64_t N, const float *__restrict__ U, int rp,
                                                 int rk, const float *__restrict__ P, int ldb,
                                                 int64_t rc, float *__restrict__ Cpart,
                                                 IterGuard ig) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    constexpr int G = 8;  // MFMA k-steps (2 rows each) per pipeline stage
    const int lane = threadIdx.x % kWave;
    const int w = threadIdx.x / kWave;
    // logical tiles: column group fastest, then k group, then row chunk, so
    // the tiles of one row chunk run on one XCD and share its rows in L2
    const unsigned L = xcd_tile(), ncg = (unsigned)ldb / (32 * NT),
                   nkg = (unsigned)(rk / 32 + 3) / 4;
    const unsigned chunk = L / (ncg * nkg);
    const int k0 = ((int)((L / ncg) % nkg) * 4 + w) * 32;
    if (k0 >= rk) return;  // no block-level synchronisation below
    const int b0 = (int)(L % ncg) * 32 * NT;
    const int64_t rs = (int64_t)chunk * rc;
    const int64_t re = rs + rc < N ? rs + rc : N;
    const int hi = lane / 32, lo = lane % 32;
    f32x16 acc[NT];
#pragma unroll
    for (int t = 0; t < NT; ++t)
        for (int v = 0; v < 16; ++v) acc[t][v] = 0.f;

    const int64_t full_end = rs + ((re - rs) / (2 * G)) * (2 * G);
    float a[G], b[G][NT];
    int64_t i = rs;
    if (i < full_end) {
#pragma unroll
        for (int u = 0; u < G; ++u) {
            const int64_t row = i + 2 * u + hi;
            a[u] = U[(size_t)row * rp + k0 + lo];
#pragma unroll
            for (int t = 0; t < NT; ++t) b[u][t] = P[vec_index(N, ldb, row, b0 + t * 32 + lo)];
        }
    }
    for (; i < full_end; i += 2 * G) {
        float an[G], bn[G][NT];
        const bool more = i + 2 * G < full_end;
        if (more) {
#pragma unroll
            for (int u = 0; u < G; ++u) {
                const int64_t row = i + 2 * G + 2 * u + hi;
                an[u] = U[(size_t)row * rp + k0 + lo];
#pragma unroll
                for (int t = 0; t < NT; ++t) bn[u][t] = P[vec_index(N, ldb, row, b0 + t * 32 + lo)];
            }
        }
#pragma unroll
        for (int u = 0; u < G; ++u)
#pragma unroll
            for (int t = 0; t < NT; ++t) acc[t] = mfma32(a[u], b[u][t], acc[t]);
        if (more) {
#pragma unroll
            for (int u = 0; u < G; ++u) {
                a[u] = an[u];
#pragma unroll
                for (int t = 0; t < NT; ++t) b[u][t] = bn[u][t];
            }
        }
    }
    for (; i < re; i += 2) {
        const int64_t row = i + hi;
        float a1 = 0.f, b1[NT];
#pragma unroll
        for (int t = 0; t < NT; ++t) b1[t] = 0.f;
        if (row < re) {
            a1 = U[(size_t)row * rp + k0 + lo];
#pragma unroll
            for (int t = 0; t < NT; ++t) b1[t] = P[vec_index(N, ldb, row, b0 + t * 32 + lo)];
        }
#pragma unroll
        for (int t = 0; t < NT; ++t) acc[t] = mfma32(a1, b1[t], acc[t]);
    }
    float *out = Cpart + (size_t)chunk * rk * ldb;
#pragma unroll
    for (int t = 0; t < NT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v)
            out[(size_t)(k0 + acc_row(v, lane)) * ldb + b0 + t * 32 + lo] = acc[t][v];
}

hipError_t launch_ut_p(int64_t N, const float *U, int rp, int rk, const float *P, int ldb,
                       float *Cpart, IterGuard g, hipStream_t s) {
    int64_t rc;
    int nchunk = ut_p_chunks(N, &rc);
    int kgroups = (rk / 32 + 3) / 4;
    if (ldb == 64) {
        k_ut_p<2><<<(unsigned)(nchunk * kgroups), kBlock, 0, s>>>(N, U, rp, rk, P, ldb, rc, Cpart, g);
    } else {
        k_ut_p<4><<<(unsigned)(nchunk * kgroups * (ldb / 128)), kBlock, 0, s>>>(N, U, rp, rk, P, ldb,
                                                                                rc, Cpart, g);
    }
    return hipGetLastError();
}

// Cl = L1 .* sum over chunks of Cpart. A block reduces 64 consecutive
// entries of the rk x ldb matrix: its four waves take the chunks c = w mod 4
// with two accumulators each, then the four wave sums are added in order.
__global__ __launch_bounds__(kBlock) void k_reduce_c(int nchunk, const float *__restrict__ Cpart,
                                                     int rk, int ldb, const double *lam, int r_use,
                                                     float *__restrict__ Cl, IterGuard ig,
                                                     double *__restrict__ Dg, double cc,
                                                     const float *__restrict__ uscale) {
    if (all_stopped(ig.nact, ig.ntile)) return;
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
        const int k = (int)(idx / ldb);
        // fp8 codes: the scale of component k turns the codes' product into
        // U1^T P, and once more makes Cl the coefficient of the codes
        const double sk = uscale && k < r_use ? (double)uscale[k] : 1.0;
        const double sum = (((sh[0][lane] + sh[1][lane]) + sh[2][lane]) + sh[3][lane]) * sk;
        Cl[idx] = k < r_use ? (float)(lam[k] * sum * sk) : 0.f;
        if (Dg) Dg[idx] = k < r_use ? cc * lam[k] * sum * sum : 0.0;
    }
}

hipError_t launch_reduce_c(int nchunk, const float *Cpart, int rk, int ldb, const double *lam,
                           int r_use, float *Cl, IterGuard g, hipStream_t s, double *Dg, double alpha,
                           const float *uscale) {
    size_t tot = (size_t)rk * ldb;
    const double cc = Dg ? alpha / (1.0 - alpha) : 0.0;
    k_reduce_c<<<(unsigned)(tot / kWave), kBlock, 0, s>>>(nchunk, Cpart, rk, ldb, lam, r_use, Cl, g, Dg, cc,
                                                          uscale);
    return hipGetLastError();
}

// Operand staging shared by u_c and combine. A block covers 128 rows; per
// 32-wide k chunk it holds U[128 rows][32 k] and C[32 k][64*NT columns] in
// LDS. The next chunk is fetched into registers (float4) while the MFMAs of
// the current chunk run, then written to LDS between two barriers.
template <int NT>
struct UcStage {
    static constexpr int ROWS = 128;
    static constexpr int COLS = 64 * NT;
    float4 u[4];       // U: thread t -> row t/2, k (t%2)*16 .. +16
    float4 c[2 * NT];  // C: float4 index t + 256 m of the 32 x COLS chunk

    __device__ __forceinline__ void fetch(const float *__restrict__ U, int rp, int64_t N,
                                          int64_t i0, int k0, const float *__restrict__ C,
                                          int ldb, int c0) {
        const int t = threadIdx.x;
        const int64_t gi = i0 + t / 2;
        const int kk = (t % 2) * 16;
        if (gi < N) {
            const float4 *src = reinterpret_cast<const float4 *>(U + (size_t)gi * rp + k0 + kk);
#pragma unroll
            for (int m = 0; m < 4; ++m) u[m] = src[m];
        } else {
#pragma unroll
            for (int m = 0; m < 4; ++m) u[m] = make_float4(0.f, 0.f, 0.f, 0.f);
        }
#pragma unroll
        for (int m = 0; m < 2 * NT; ++m) {
            const int f = t + kBlock * m;
            const int kr = f / (COLS / 4), c4 = (f % (COLS / 4)) * 4;
            c[m] = *reinterpret_cast<const float4 *>(C + (size_t)(k0 + kr) * ldb + c0 + c4);
        }
    }
    __device__ __forceinline__ void store(float (*Us)[33], float (*Cs)[COLS + 4]) const {
        const int t = threadIdx.x;
        const int row = t / 2, kk = (t % 2) * 16;
#pragma unroll
        for (int m = 0; m < 4; ++m) {
            Us[row][kk + 4 * m + 0] = u[m].x;
            Us[row][kk + 4 * m + 1] = u[m].y;
            Us[row][kk + 4 * m + 2] = u[m].z;
            Us[row][kk + 4 * m + 3] = u[m].w;
        }
#pragma unroll
        for (int m = 0; m < 2 * NT; ++m) {
            const int f = t + kBlock * m;
            const int kr = f / (COLS / 4), c4 = (f % (COLS / 4)) * 4;
            *reinterpret_cast<float4 *>(&Cs[kr][c4]) = c[m];
        }
    }
};

// acc[t] (t < 2*NT) += U[rows 32w..32w+31] x C[:, 32t..32t+31] over one chunk.
template <int NT>
__device__ __forceinline__ void uc_chunk(const float (*Us)[33], const float (*Cs)[64 * NT + 4],
                                         f32x16 *acc) {
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int hi = lane / 32, lo = lane % 32;
#pragma unroll 4
    for (int kk = 0; kk < 32; kk += 2) {
        const float a = Us[32 * w + lo][kk + hi];
#pragma unroll
        for (int t = 0; t < 2 * NT; ++t) acc[t] = mfma32(a, Cs[kk + hi][32 * t + lo], acc[t]);
    }
}

// Z = P + alpha U Cl for 128 rows x 64*NT columns; wave w owns rows
// 32w..32w+31 and all the block's columns.
template <int NT>
__global__ __launch_bounds__(kBlock) void k_u_c(int64_t N, const float *__restrict__ U, int rp,
                                                int rk, const float *__restrict__ Cl, int ldb,
                                                const float *__restrict__ P, float alpha,
                                                float *__restrict__ Z, IterGuard ig) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    constexpr int COLS = 64 * NT;
    __shared__ float Us[128][33];
    __shared__ __attribute__((aligned(16))) float Cs[32][COLS + 4];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int lo = lane % 32;
    // logical tiles: column group fastest, then 128-row block
    const unsigned L = xcd_tile(), ncg = (unsigned)ldb / COLS;
    const int64_t i0 = (int64_t)(L / ncg) * 128;
    const int c0 = (int)(L % ncg) * COLS;
    f32x16 acc[2 * NT];
#pragma unroll
    for (int t = 0; t < 2 * NT; ++t)
        for (int v = 0; v < 16; ++v) acc[t][v] = 0.f;
    UcStage<NT> st;
    if (rk > 0) st.fetch(U, rp, N, i0, 0, Cl, ldb, c0);
    for (int k0 = 0; k0 < rk; k0 += 32) {
        __syncthreads();
        st.store(Us, Cs);
        __syncthreads();
        if (k0 + 32 < rk) st.fetch(U, rp, N, i0, k0 + 32, Cl, ldb, c0);
        uc_chunk<NT>(Us, Cs, acc);
    }
#pragma unroll
    for (int t = 0; t < 2 * NT; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int64_t i = i0 + 32 * w + acc_row(v, lane);
            if (i < N) {
                const size_t o = vec_index(N, ldb, i, c0 + 32 * t + lo);
                Z[o] = P[o] + alpha * acc[t][v];
            }
        }
}

hipError_t launch_u_c(int64_t N, const float *U, int rp, int rk, const float *Cl, int ldb,
                      const float *P, double alpha, float *Z, IterGuard g, hipStream_t s) {
    const unsigned gx = (unsigned)((N + 127) / 128);
    if (ldb == 64) {
        k_u_c<1><<<gx, kBlock, 0, s>>>(N, U, rp, rk, Cl, ldb, P, (float)alpha, Z, g);
    } else if (ldb == 128) {
        k_u_c<2><<<gx, kBlock, 0, s>>>(N, U, rp, rk, Cl, ldb, P, (float)alpha, Z, g);
    } else {
        k_u_c<4><<<gx * (unsigned)(ldb / 256), kBlock, 0, s>>>(N, U, rp, rk, Cl, ldb, P, (float)alpha,
                                                                 Z, g);
    }
    return hipGetLastError();
}

// x[b][i] = (U Cs)[i][b] + X[i][b] for 128 items x 64 queries per block: the
// product is formed as in u_c, the temporal term added in the accumulator
// layout, and the tile transposed through LDS so that each query's 128 items
// are written as one contiguous run.
__global__ __launch_bounds__(kBlock) void k_combine(int64_t N, int B, const float *__restrict__ U,
                                                    int rp, int rk, const float *__restrict__ Csp,
                                                    int ldb, const float *__restrict__ X,
                                                    float *__restrict__ x, int64_t ldx,
                                                    const int32_t *__restrict__ gate) {
    if (gate && *gate == 0) return;
    __shared__ float Us[128][33];
    __shared__ __attribute__((aligned(16))) float Cs[32][64 + 4];
    __shared__ float T[64][129];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int lo = lane % 32;
    // logical tiles: 64-query group fastest, then 128-row block
    const unsigned L = xcd_tile(), nqg = (unsigned)(B + 63) / 64;
    const int64_t i0 = (int64_t)(L / nqg) * 128;
    const int c0 = (int)(L % nqg) * 64;
    f32x16 acc[2];
    for (int v = 0; v < 16; ++v) {
        acc[0][v] = 0.f;
        acc[1][v] = 0.f;
    }
    UcStage<1> st;
    if (rk > 0) st.fetch(U, rp, N, i0, 0, Csp, ldb, c0);
    for (int k0 = 0; k0 < rk; k0 += 32) {
        __syncthreads();
        st.store(Us, Cs);
        __syncthreads();
        if (k0 + 32 < rk) st.fetch(U, rp, N, i0, k0 + 32, Csp, ldb, c0);
        uc_chunk<1>(Us, Cs, acc);
    }
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
        for (int v = 0; v < 16; ++v) {
            const int rl = 32 * w + acc_row(v, lane);
            const int64_t i = i0 + rl;
            const int bl = 32 * t + lo;
            float val = acc[t][v];
            if (i < N) val += X[vec_index(N, ldb, i, c0 + bl)];
            T[bl][rl] = val;
        }
    __syncthreads();
    for (int f = threadIdx.x; f < 64 * 128; f += kBlock) {
        const int bl = f / 128, rl = f % 128;
        const int b = c0 + bl;
        const int64_t i = i0 + rl;
        if (b < B && i < N) x[(size_t)b * ldx + i] = T[bl][rl];
    }
}

// x[b][i] = X[i][b] (the combine with no eigenvector term): a block
// transposes a 64-item x 64-query tile through LDS, reading 256-byte runs of
// X's rows and writing 256-byte runs of x's rows.
// FOLD: x + a p (XFold), loads of X and P issued together.
template <bool FOLD>
__global__ __launch_bounds__(kBlock) void k_xt(int64_t N, int B, int ldb, const float *__restrict__ X,
                                               float *__restrict__ x, int64_t ldx,
                                               const int32_t *__restrict__ gate, XFold fold) {
    if (gate && *gate == 0) return;
    __shared__ float T[64][65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int b0 = blockIdx.y * 64;
    const int c = threadIdx.x % 64, r0 = threadIdx.x / 64;
    const double fa = FOLD && !all_stopped(fold.g.nact, fold.g.ntile) ? fold.a[b0 + c] : 0.0;
    float v[16], pv[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int64_t i = i0 + r0 + 4 * r;
        const size_t o = vec_index(N, ldb, i < N ? i : N - 1, b0 + c);
        v[r] = X[o];
        if (FOLD) pv[r] = fold.P[o];
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        if (FOLD) v[r] = fold_x(v[r], pv[r], fa);
        if (i0 + r0 + 4 * r >= N || b0 + c >= B) v[r] = 0.f;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) T[r0 + 4 * r][c] = v[r];
    __syncthreads();
#pragma unroll
    for (int r = 0; r < 16; ++r) {
        const int bl = r0 + 4 * r;
        const int64_t i = i0 + c;
        if (b0 + bl < B && i < N) x[(size_t)(b0 + bl) * ldx + i] = T[c][bl];
    }
}

hipError_t launch_combine(int64_t N, int B, const float *U, int rp, int rk, const float *Cs,
                          int ldb, const float *X, float *x, int64_t ldx, hipStream_t s,
                          const int32_t *gate, const XFold *fold) {
    if (rk == 0) {
        const dim3 g((unsigned)((N + 63) / 64), (unsigned)((B + 63) / 64));
        if (fold)
            k_xt<true><<<g, kBlock, 0, s>>>(N, B, ldb, X, x, ldx, gate, *fold);
        else
            k_xt<false><<<g, kBlock, 0, s>>>(N, B, ldb, X, x, ldx, gate, XFold{nullptr, nullptr, IterGuard{nullptr, 0}});
        return hipGetLastError();
    }
    if (fold) return hipErrorInvalidValue;
    const unsigned nblk = (unsigned)((N + 127) / 128) * (unsigned)((B + 63) / 64);
    k_combine<<<nblk, kBlock, 0, s>>>(N, B, U, rp, rk, Cs, ldb, X, x, ldx, gate);
    return hipGetLastError();
}

}  // namespace hd
