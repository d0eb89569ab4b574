// BF16 storage form of the eigenvector products (the precision form of the
// low-rank parts of Section 4.2, eqs. (h-spectral) and (box)).
//
// U1 is stored in bfloat16 twice: item-major (N x rp, for U C) and
// component-major (rp x N, for U^T P), each in fragment order (16 x 32
// tiles laid out as the 64 lanes' MFMA operands, frag_offset), so that a
// wave reads every A operand tile as one contiguous kilobyte. The other
// operand (P, or the small coefficient matrix C) stays fp32 in memory and is
// split into hi + lo bfloat16 parts (hi = RNE(v), lo = RNE(v - hi)); each
// product is done twice (hi and lo) into fp32 accumulators, so the only
// approximation beyond fp32 is the bfloat16 storage of U1 itself.
//
// Two-term form (AK_BF16X2): U1 is also stored as U_hi + U_lo, two bfloat16
// arrays of the same layout (about 16 significant bits), and each product
// takes the three terms U_hi P_hi + U_hi P_lo + U_lo P_hi (the U_lo P_lo term
// is below fp32 rounding of the sum and is dropped).
//
// FP8 form: U1 is stored as OCP FP8 E4M3 codes in the same fragment order
// (one byte per element, so a wave's operand tile is half a kilobyte) with
// one fp32 scale per component. Each lane converts its eight codes to
// bfloat16 in registers (exact: every E4M3 value is a bfloat16 value) and
// the products run as in the one-term form; the scales are applied to the
// small coefficient matrices by the callers.
//
// MFMA v_mfma_f32_16x16x32_bf16 operand layout (lane l of 64):
//   A (16 x 32): row l % 16, k = 8*(l/16) .. +7;  B (32 x 16): col l % 16,
//   k = 8*(l/16) .. +7;  C (16 x 16, 4 values): row 4*(l/16) + v, col l % 16.
#include "hd_device.h"
#include "hd_kernels.h"
#include "hd_emit.h"

namespace hd {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mfma16bf(bf16x8 a, bf16x8 b, f32x4 c) {
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// fp32 -> bf16 bits, round to nearest even (the gfx950 conversion
// instruction v_cvt_pk_bf16_f32).
__device__ __forceinline__ unsigned short bf16_rne(float x) {
    return __builtin_bit_cast(unsigned short, (__bf16)x);
}
__device__ __forceinline__ float bf16_to_f(unsigned short h) {
    return __uint_as_float((uint32_t)h << 16);
}
__device__ __forceinline__ bf16x8 load8(const unsigned short *p) {
    return __builtin_bit_cast(bf16x8, *reinterpret_cast<const u16x8 *>(p));
}

// Eight OCP FP8 E4M3 codes (consecutive bytes, element 0 in the lowest
// byte) to eight bfloat16 values by the gfx950 scaled conversion with scale
// 1, two codes per instruction.
typedef __bf16 bf16x2v __attribute__((ext_vector_type(2)));
__device__ __forceinline__ bf16x8 fp8x8_to_bf16(uint2 w) {
    const bf16x2v a = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w.x, 1.0f, false);
    const bf16x2v b = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w.x, 1.0f, true);
    const bf16x2v c = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w.y, 1.0f, false);
    const bf16x2v d = __builtin_amdgcn_cvt_scalef32_pk_bf16_fp8(w.y, 1.0f, true);
    return bf16x8{a[0], a[1], b[0], b[1], c[0], c[1], d[0], d[1]};
}

// Storage kinds of the streamed operand: one bfloat16 term, two terms
// (hi + lo), FP8 E4M3 codes.
enum { AK_BF16 = 0, AK_BF16X2 = 1, AK_FP8 = 2 };
// The eight consecutive elements of a lane's operand piece at element offset
// o (a multiple of 8) of a stored operand of kind AK.
template <int AK>
__device__ __forceinline__ bf16x8 load_a8(const void *A, size_t o) {
    if (AK == AK_FP8) return fp8x8_to_bf16(*reinterpret_cast<const uint2 *>(reinterpret_cast<const uint8_t *>(A) + o));
    return load8(reinterpret_cast<const unsigned short *>(A) + o);
}
static inline int akind(const UOperand &u) { return u.fp8 ? AK_FP8 : (u.lo ? AK_BF16X2 : AK_BF16); }

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
    // idx runs over CT in fragment order (kt = rk / 32 tiles per tile row)
    const int kt = rk / 32, e = (int)(idx % 8), l = (int)((idx / 8) % 64);
    const size_t tile = idx / 512;
    const int b = (int)(tile / kt) * 16 + l % 16, k = (int)(tile % kt) * 32 + 8 * (l / 16) + e;
    const float v = C[(size_t)k * ldb + b];
    const unsigned short h = bf16_rne(v);
    CT_hi[idx] = h;
    CT_lo[idx] = bf16_rne(v - bf16_to_f(h));
}

hipError_t launch_split_t(const float *C, int rk, int ldb, unsigned short *CT_hi,
                          unsigned short *CT_lo, IterGuard g, hipStream_t s) {
    const size_t tot = (size_t)rk * ldb;
    if (tot == 0) return hipSuccess;
    if (rk % 32 != 0 || ldb % 16 != 0) return hipErrorInvalidValue;  // whole fragment tiles
    k_split_t<<<(unsigned)((tot + kBlock - 1) / kBlock), kBlock, 0, s>>>(C, rk, ldb, CT_hi, CT_lo, g);
    return hipGetLastError();
}

// m-tiles per wave of the block GEMM for NT n-tiles per wave
constexpr int tn_mt(int nt) { return nt == 4 ? 2 : 4; }
// rows of M per block
constexpr int tn_rows(int nt) { return 64 * tn_mt(nt); }
static inline int tn_rows_rt(int nt) { return nt == 4 ? tn_rows(4) : tn_rows(1); }

// ---------------------------------------------------------------------------
// Block GEMM shared by the three eigenvector products:
//   acc[m][n] = sum_k A[m][k] B[n][k]
// with both operands K-contiguous bfloat16: A (M x K in fragment order, kt
// tiles of 32 K per 16-row tile row, rows padded to a multiple of 16; one or
// two terms A + Al) and B (N x K in fragment order, ktb tiles per tile row,
// split hi + lo). A block
// covers 64 MT rows of M and 64*NT columns of N (from nb0); wave w owns rows
// m0 + 16 MT w .. +16 MT - 1 (MT m-tiles) for all 64 NT columns (4 NT
// n-tiles), so it holds 4 MT NT accumulators per lane. MT = 4 (NT <= 2) or 2
// (NT = 4, to stay within the registers of two waves per SIMD): each B
// fragment read from LDS feeds 3 MT MFMAs. A is the large streamed operand (U1): each
// wave loads its own A fragments straight from global memory into registers,
// one 32-wide K step ahead, with no LDS staging and no barrier between the
// load and its use; in fragment order each of those loads is one contiguous
// kilobyte per wave (with rows of a plain row-major A it touched sixteen
// rows and measured 1.2-2x slower). B (the coefficients, or the split P^T) is shared by the
// four waves: per K step the block loads the 64 NT x 32 B tile - 4 NT
// fragment tiles of a kilobyte, hi and lo - once (NT 16-byte pieces per
// thread, each wave copying whole tiles), stages it in LDS in the same order
// and every wave reads its B fragments there; the next step's B pieces are
// fetched into registers while the current step's MFMAs run.
//   products per (A term, B term): A_hi B_hi + A_hi B_lo (+ A_lo B_hi)
// The accumulation order over K (and of the terms) is fixed: results do not
// depend on NT.
// MFMA v_mfma_f32_16x16x32_bf16: A fragment = A[m0 + l%16][k + 8(l/16) ..+7],
// B fragment = B[n + l%16][k + 8(l/16) ..+7], C[m = 4(l/16) + v][n = l%16].
// In fragment order a wave's B fragment read from LDS is one contiguous
// kilobyte, lane l at 16 l bytes, so it is free of bank conflicts.
template <int AK, int NT, int MT = tn_mt(NT)>
__device__ __forceinline__ void tn_block(const void *__restrict__ A,
                                         const void *__restrict__ Al, int64_t kt,
                                         int64_t m0, int64_t mend,
                                         const unsigned short *__restrict__ Bh,
                                         const unsigned short *__restrict__ Bl, int64_t ktb,
                                         int64_t nb0, int64_t k0, int64_t k1, f32x4 (&acc)[MT][4 * NT]) {
    __shared__ __attribute__((aligned(16))) unsigned short Bsh[4 * NT][512];
    __shared__ __attribute__((aligned(16))) unsigned short Bsl[4 * NT][512];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int g = lane / 16, c16 = lane % 16;
    // this lane's place in its A tiles (one tile row per m-tile); K step k
    // is tile k / 32 of the row, 512 elements on. Every load is
    // unconditional and in bounds: a tile past the last row tile reads tile
    // m0 / 16 instead (its accumulator rows are never stored; rows past mend
    // inside the last tile are the zero padding), and a K step past k1
    // reloads the last step (never used). Loads without branches keep the
    // compiler's wait counts exact, so waiting for the staged B pieces does
    // not also wait for the A prefetch issued after them.
    constexpr bool LO = AK == AK_BF16X2;
    size_t pa[MT];  // element offsets of this lane's pieces (bytes for fp8 codes)
    const int64_t mtiles = (mend + 15) / 16;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int64_t tb = m0 / 16 + MT * w + mt;
        pa[mt] = ((size_t)(tb < mtiles ? tb : m0 / 16) * (size_t)kt * 64 + (size_t)lane) * 8;
    }
    const int64_t klast = k1 - 32;  // the last K step (K ranges are multiples of 32)
    // B staging: wave w copies lane `lane` of the block's n-tiles w, w + 4,
    // ... (tile rows nb0 / 16 + w + 4 j, j < NT), four tile rows apart
    const size_t boff = ((size_t)(nb0 / 16 + w) * (size_t)ktb * 64 + (size_t)lane) * 8;
    const unsigned short *sbh = Bh + boff;
    const unsigned short *sbl = Bl + boff;
    const size_t bstep = (size_t)4 * (size_t)ktb * 512;
    bf16x8 af[2][MT], afl[2][MT], rbh[NT], rbl[NT];
    auto fetch_a = [&](int slot, int64_t k) {
        const int64_t kc = k < k1 ? k : klast;
#pragma unroll
        for (int mt = 0; mt < MT; ++mt) {
            af[slot][mt] = load_a8<AK>(A, pa[mt] + (size_t)kc * 16);  // tile kc / 32, 512 apart
            if (LO) afl[slot][mt] = load_a8<AK_BF16>(Al, pa[mt] + (size_t)kc * 16);
        }
    };
    auto fetch_b = [&](int64_t k) {
        const int64_t kc = k < k1 ? k : klast;
#pragma unroll
        for (int j = 0; j < NT; ++j) {
            rbh[j] = load8(sbh + j * bstep + (size_t)kc * 16);
            rbl[j] = load8(sbl + j * bstep + (size_t)kc * 16);
        }
    };
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int n = 0; n < 4 * NT; ++n) acc[mt][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    if (k0 >= k1) return;
    fetch_a(0, k0);
    fetch_b(k0);
    // two K steps per trip so that the A register slots have fixed names
    for (int64_t k = k0; k < k1; k += 64) {
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            const int64_t kk = k + 32 * st;
            if (kk < k1) {
                __syncthreads();  // the previous step's LDS reads are done
#pragma unroll
                for (int j = 0; j < NT; ++j) {
                    *reinterpret_cast<bf16x8 *>(&Bsh[w + 4 * j][8 * lane]) = rbh[j];
                    *reinterpret_cast<bf16x8 *>(&Bsl[w + 4 * j][8 * lane]) = rbl[j];
                }
                __syncthreads();
                fetch_b(kk + 32);
                fetch_a(st ^ 1, kk + 32);
#pragma unroll
                for (int n = 0; n < 4 * NT; ++n) {
                    const bf16x8 bh = load8(&Bsh[n][8 * lane]);
                    const bf16x8 bl = load8(&Bsl[n][8 * lane]);
#pragma unroll
                    for (int mt = 0; mt < MT; ++mt) {
                        acc[mt][n] = mfma16bf(af[st][mt], bh, acc[mt][n]);
                        acc[mt][n] = mfma16bf(af[st][mt], bl, acc[mt][n]);
                        if (LO) acc[mt][n] = mfma16bf(afl[st][mt], bh, acc[mt][n]);
                    }
                }
            }
        }
    }
}

// Number of n-tiles per wave (columns per block: 64 NT): the requested
// value, or by default the widest of 1, 2, 4 up to `cap` that divides ldb
// (measured defaults: 4 for U^T P, 2 for U C, whose four-tile form holds one
// wave per SIMD).
static inline int tn_nt(int ldb, int req, int cap) {
    if (req != 0) return tile_param_ok(req, ldb) ? req : 0;
    for (int v = cap; v > 1; v /= 2)
        if (ldb % (64 * v) == 0) return v;
    return 1;
}

// ---------------------------------------------------------------------------
// P^T split: from P (N x ldb fp32, node-major) write PT_hi, PT_lo (ldb x ldpt
// bfloat16 in fragment order over items; items N .. ldpt-1 zero), the B
// operand of U^T P. A block transposes a 64-item x 64-column tile through LDS.
__global__ __launch_bounds__(kBlock) void k_split_pt(int64_t N, int ldb, const float *__restrict__ P,
                                                     int64_t ldpt, unsigned short *__restrict__ PTh,
                                                     unsigned short *__restrict__ PTl, IterGuard ig) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    __shared__ float T[64][65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int b0 = blockIdx.y * 64;
    const int c = threadIdx.x % 64;
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        const int r = threadIdx.x / 64 + 4 * j;
        T[c][r] = i0 + r < N ? P[vec_index(N, ldb, i0 + r, b0 + c)] : 0.f;
    }
    __syncthreads();
    const int b = threadIdx.x / 4, seg = 16 * (threadIdx.x % 4);
    bf16x8 h[2], l[2];
#pragma unroll
    for (int u = 0; u < 2; ++u)
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            const float v = T[b][seg + 8 * u + q];
            const __bf16 hb = (__bf16)v;
            h[u][q] = hb;
            l[u][q] = (__bf16)(v - (float)hb);
        }
    // PT in fragment order: each run of 8 items is one 16-byte lane piece
#pragma unroll
    for (int u = 0; u < 2; ++u) {
        const size_t o = frag_offset(b0 + b, i0 + seg + 8 * u, ldpt / 32);
        *reinterpret_cast<bf16x8 *>(PTh + o) = h[u];
        *reinterpret_cast<bf16x8 *>(PTl + o) = l[u];
    }
}

hipError_t launch_split_pt(int64_t N, int ldb, const float *P, int64_t ldpt, unsigned short *PTh,
                           unsigned short *PTl, IterGuard g, hipStream_t s, int width) {
    if (width == 0) width = ldb;
    if (ldpt % 64 != 0 || ldpt < N || ldb % 64 != 0 || width % 64 != 0 || width > ldb)
        return hipErrorInvalidValue;
    k_split_pt<<<dim3((unsigned)(ldpt / 64), (unsigned)(width / 64)), kBlock, 0, s>>>(N, ldb, P, ldpt, PTh,
                                                                                    PTl, g);
    return hipGetLastError();
}

// Admitted columns: zero their lane pieces, then write the split of P at
// their y rows. Zeroing: thread -> (slot t = 32 y + tid % 32, piece
// 8 x + tid / 32) with the slot fastest, so adjacent admitted columns (the
// usual case) write adjacent 16-byte pieces of one fragment tile.
__global__ __launch_bounds__(kBlock) void k_pt_zero_cols(const int32_t *__restrict__ cols, int ncols,
                                                         int64_t ldpt, unsigned short *__restrict__ PTh,
                                                         unsigned short *__restrict__ PTl) {
    const int t = (int)blockIdx.y * 32 + (int)threadIdx.x % 32;
    const int64_t p = (int64_t)blockIdx.x * (kBlock / 32) + threadIdx.x / 32;
    if (t >= ncols || p >= ldpt / 8) return;
    const size_t o = frag_offset(cols[t], 8 * p, ldpt / 32);
    *reinterpret_cast<uint4 *>(PTh + o) = make_uint4(0u, 0u, 0u, 0u);
    *reinterpret_cast<uint4 *>(PTl + o) = make_uint4(0u, 0u, 0u, 0u);
}

__global__ __launch_bounds__(kBlock) void k_pt_scatter_y(int m, int ky, const int32_t *__restrict__ ids,
                                                         const int32_t *__restrict__ cols, int64_t N, int ldb,
                                                         const float *__restrict__ P, int64_t ldpt,
                                                         unsigned short *__restrict__ PTh,
                                                         unsigned short *__restrict__ PTl) {
    const int t = blockIdx.x * kBlock + threadIdx.x;
    if (t >= m * ky) return;
    const int64_t i = ids[t];
    if (i < 0 || i >= N) return;  // the admission's id check rejects the batch
    const int col = cols[t / ky];
    // repeated ids write the same value (P holds their sum)
    const float v = P[vec_index(N, ldb, i, col)];
    const __bf16 hb = (__bf16)v;
    const size_t o = frag_offset(col, i, ldpt / 32);
    PTh[o] = __builtin_bit_cast(unsigned short, hb);
    PTl[o] = __builtin_bit_cast(unsigned short, (__bf16)(v - (float)hb));
}

hipError_t launch_pt_admit(int m, int ky, const int32_t *ids, const int32_t *cols, const int32_t *zcols, int nz,
                           int64_t N, int ldb, const float *P, int64_t ldpt, unsigned short *PTh,
                           unsigned short *PTl, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    if (ldpt % 64 != 0 || ldpt < N || ky < 1 || nz < 0) return hipErrorInvalidValue;
    if (nz > 0) {
        const int64_t pieces = ldpt / 8, per = kBlock / 32;
        k_pt_zero_cols<<<dim3((unsigned)((pieces + per - 1) / per), (unsigned)((nz + 31) / 32)), kBlock, 0, s>>>(
            zcols, nz, ldpt, PTh, PTl);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int tot = m * ky;
    k_pt_scatter_y<<<(unsigned)((tot + kBlock - 1) / kBlock), kBlock, 0, s>>>(m, ky, ids, cols, N, ldb, P, ldpt, PTh,
                                                                           PTl);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Cpart[c] = U[chunk c]^T P[chunk c]: M = k (UT rows, component-major U,
// row stride ldut, items past N zero), N = b (PT rows), K = the chunk's
// items. Logical tiles: column group fastest, then k group, then row chunk,
// so the tiles of one chunk run on one XCD and share PT and UT in its L2.
template <int AK, int NT>
__global__ __launch_bounds__(kBlock, 2) void k_ut_p_tn(const void *__restrict__ UT,
                                                    const void *__restrict__ UTl,
                                                    int64_t ldut, int rk,
                                                    const unsigned short *__restrict__ PTh,
                                                    const unsigned short *__restrict__ PTl, int ldb,
                                                    int wcols, int64_t rc, int64_t kend_all,
                                                    float *__restrict__ Cpart, IterGuard ig) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    constexpr int MT = tn_mt(NT), RB = tn_rows(NT);
    const unsigned L = xcd_tile(), ncg = (unsigned)wcols / (64 * NT), nkg = (unsigned)(rk + RB - 1) / RB;
    const unsigned chunk = L / (ncg * nkg);
    const int64_t m0 = (int64_t)((L / ncg) % nkg) * RB;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t nb0 = (int64_t)(L % ncg) * 64 * NT;
    const int64_t ks = (int64_t)chunk * rc;
    const int64_t ke = ks + rc < kend_all ? ks + rc : kend_all;
    f32x4 acc[MT][4 * NT];
    tn_block<AK, NT>(UT, UTl, ldut / 32, m0, rk, PTh, PTl, ldut / 32, nb0, ks, ke, acc);
    float *out = Cpart + (size_t)chunk * rk * ldb;
    const int g = lane / 16, c16 = lane % 16;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t k = m0 + 16 * MT * w + 16 * mt + 4 * g + v;
            if (k >= rk) continue;
#pragma unroll
            for (int n = 0; n < 4 * NT; ++n) out[(size_t)k * ldb + nb0 + 16 * n + c16] = acc[mt][n][v];
        }
}

hipError_t launch_ut_p_bf16(int64_t N, UOperand UT, int64_t ldut, int rk, const unsigned short *PTh, const unsigned short *PTl,
                            int ldb, float *Cpart, IterGuard g, hipStream_t s, int ntr, int width) {
    int64_t rc;
    const int nchunk = ut_p_chunks(N, &rc);
    // rows run to N rounded up to 32 (UT and PT are zero past N)
    const int64_t kend = (N + 31) / 32 * 32;
    if (width == 0) width = ldb;
    if (kend > ldut || rc % 32 != 0 || width % 64 != 0 || width > ldb) return hipErrorInvalidValue;
    const int nt = tn_nt(width, ntr, 4);
    if (nt == 0) return hipErrorInvalidValue;
    const unsigned nblk = (unsigned)(width / (64 * nt)) * (unsigned)((rk + tn_rows_rt(nt) - 1) / tn_rows_rt(nt)) *
                          (unsigned)nchunk;
#define HD_UTP(AKV, NTV)                                                                                     \
    k_ut_p_tn<AKV, NTV><<<nblk, kBlock, 0, s>>>(UT.hi, UT.lo ? UT.lo : UT.hi, ldut, rk, PTh, PTl, ldb, width, rc, \
                                                kend, Cpart, g)
#define HD_UTP_NT(AKV) \
    if (nt == 4) HD_UTP(AKV, 4); else if (nt == 2) HD_UTP(AKV, 2); else HD_UTP(AKV, 1)
    switch (akind(UT)) {
        case AK_FP8: HD_UTP_NT(AK_FP8); break;
        case AK_BF16X2: HD_UTP_NT(AK_BF16X2); break;
        default: HD_UTP_NT(AK_BF16); break;
    }
#undef HD_UTP_NT
#undef HD_UTP
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Z = P + alpha U Cl: M = items (128 per block), N = solver columns, K = rk;
// A = U item-major (row stride rp), B = ClT split (ldb x rk). Logical tiles:
// column group fastest, then 128-row block.
template <int AK, int NT>
__global__ __launch_bounds__(kBlock, 2) void k_u_c_tn(int64_t N, const void *__restrict__ U,
                                                   const void *__restrict__ Ul, int rp, int rk,
                                                   const unsigned short *__restrict__ CT_hi,
                                                   const unsigned short *__restrict__ CT_lo, int ldb,
                                                   const float *__restrict__ P, float alpha,
                                                   float *__restrict__ Z, IterGuard ig) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    const unsigned L = xcd_tile(), ncg = (unsigned)ldb / (64 * NT);
    constexpr int MT = tn_mt(NT), RB = tn_rows(NT);
    const int64_t i0 = (int64_t)(L / ncg) * RB;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t nb0 = (int64_t)(L % ncg) * 64 * NT;
    f32x4 acc[MT][4 * NT];
    tn_block<AK, NT>(U, Ul, rp / 32, i0, N, CT_hi, CT_lo, rk / 32, nb0, 0, rk, acc);
    const int g = lane / 16, c16 = lane % 16;
    // branch-free loads (rows past N read row N - 1 and store nothing)
#pragma unroll
    for (int mt = 0; mt < MT; ++mt)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
            const int64_t i = i0 + 16 * MT * w + 16 * mt + 4 * g + v;
            const int64_t ic = i < N ? i : N - 1;
            float pv[4 * NT];
#pragma unroll
            for (int n = 0; n < 4 * NT; ++n) pv[n] = P[vec_index(N, ldb, ic, (int)(nb0 + 16 * n + c16))];
            if (i < N) {
#pragma unroll
                for (int n = 0; n < 4 * NT; ++n)
                    Z[vec_index(N, ldb, i, (int)(nb0 + 16 * n + c16))] = pv[n] + alpha * acc[mt][n][v];
            }
        }
}

hipError_t launch_u_c_bf16(int64_t N, UOperand U, int rp, int rk,
                           const unsigned short *CT_hi, const unsigned short *CT_lo, int ldb,
                           const float *P, double alpha, float *Z, IterGuard g, hipStream_t s,
                           int ntr) {
    if (rp % 32 != 0 || rk % 32 != 0) return hipErrorInvalidValue;  // whole 32-wide K tiles
    const int nt = tn_nt(ldb, ntr, 2);
    if (nt == 0) return hipErrorInvalidValue;
    const unsigned nblk = (unsigned)(ldb / (64 * nt)) * (unsigned)((N + tn_rows_rt(nt) - 1) / tn_rows_rt(nt));
    const float a = (float)alpha;
#define HD_UC(AKV, NTV) \
    k_u_c_tn<AKV, NTV><<<nblk, kBlock, 0, s>>>(N, U.hi, U.lo ? U.lo : U.hi, rp, rk, CT_hi, CT_lo, ldb, P, a, Z, g)
#define HD_UC_NT(AKV) \
    if (nt == 4) HD_UC(AKV, 4); else if (nt == 2) HD_UC(AKV, 2); else HD_UC(AKV, 1)
    switch (akind(U)) {
        case AK_FP8: HD_UC_NT(AK_FP8); break;
        case AK_BF16X2: HD_UC_NT(AK_BF16X2); break;
        default: HD_UC_NT(AK_BF16); break;
    }
#undef HD_UC_NT
#undef HD_UC
    return hipGetLastError();
}

constexpr int kUcrMt = 2;  // m-tiles per wave of the fused residual update

// The eigenvector correction applied after the sparse product, fused with the
// CG residual update. With Qs = (P - alpha S P) / (1 - alpha) from the sparse
// product, the deflated operator gives Q = Qs + c U Cl, c = alpha / (1 - alpha)
// (Section 4.2, eq. (box)); Q is used once, in r -= a Q, so it is never
// stored: each element of the U Cl tile goes straight into the update of r,
// which follows update_r (double arithmetic, a = 0 leaves a stopped column
// untouched), and the column sums of r^2 go to part, one row of ldb doubles
// per 128-row group (a block covers one or two groups). rowmask (the first
// CG iteration, R zeroed only on the rows of y): r is taken as zero outside
// it (whatever the memory holds); every row is written.
template <int AK, int NT, bool MASKR, int MT = kUcrMt>
__global__ __launch_bounds__(kBlock, 2) void k_uc_update_r_tn(int64_t N, const void *__restrict__ U,
                                                           const void *__restrict__ Ul, int rp, int rk,
                                                           const unsigned short *__restrict__ CT_hi,
                                                           const unsigned short *__restrict__ CT_lo, int ldb,
                                                           const float *__restrict__ Qs, float cc,
                                                           float *__restrict__ R, const double *__restrict__ a,
                                                           double *__restrict__ part, int wcols, IterGuard ig,
                                                           const uint32_t *__restrict__ rowmask,
                                                           const int32_t *__restrict__ iters,
                                                           const int32_t *__restrict__ maxit) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    // two m-tiles per wave (three waves per SIMD): four measured no faster
    // in the CG iteration (1.67 against 1.66 ms a launch at 1M rows, 256
    // columns; 12% faster alone on inputs just copied in, where the
    // epilogue's loads find fewer of Qs and r in the caches)
    constexpr int RB = 64 * MT;
    const unsigned L = xcd_tile(), ncg = (unsigned)wcols / (64 * NT);
    const int64_t rb = (int64_t)(L / ncg);
    const int64_t i0 = rb * RB;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t nb0 = (int64_t)(L % ncg) * 64 * NT;
    // iters / maxit (a server's running solve): bit n set when this lane's
    // column of n-tile n ends by its cap in this iteration; its new residual
    // still enters r^2 (the stopping test and relres) but is stored as zero,
    // as nothing reads it again, so the column's r is clear for the next
    // request admitted into it
    uint32_t zmask = 0u;
    if (iters) {
#pragma unroll
        for (int n = 0; n < 4 * NT; ++n) {
            const int col = (int)(nb0 + 16 * n + lane % 16);
            zmask |= (iters[col] + 1 >= maxit[col] ? 1u : 0u) << n;
        }
    }
    f32x4 acc[MT][4 * NT];
    tn_block<AK, NT, MT>(U, Ul, rp / 32, i0, N, CT_hi, CT_lo, rk / 32, nb0, 0, rk, acc);
    const int g = lane / 16, c16 = lane % 16;
    // r^2 of each 16-row m-tile and column (4 rows per lane, then across the
    // lane groups), summed below over the m-tiles of each 128-row group in
    // order: the same sums whatever the block shape
    __shared__ double sh[4 * MT][64 * NT];
    // Per m-tile and group of up to eight n-tiles, every load of Qs and r is
    // issued before the first store to r: a store could alias a later load,
    // so loads placed after it would each wait a full memory latency.
    // Branch-free: rows past N load row N - 1 and store nothing.
    constexpr int NG = 4 * NT < 8 ? 4 * NT : 8;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
    // the first iteration's row mask: this lane's four rows (4g .. 4g + 3
    // of a 16-row m-tile, so within one 32-row mask word) read once per
    // m-tile; the mask is a separate instantiation, since a test inside the
    // load loop below, even an always-true one, split its group of loads
    // (9% slower)
    bool live[4] = {true, true, true, true};
    if (MASKR) {
        const int64_t ib = i0 + 16 * MT * w + 16 * mt + 4 * g;
        const int64_t ibc = ib < N ? ib : N - 1;
        const uint32_t word = rowmask[ibc >> 5];
#pragma unroll
        for (int v = 0; v < 4; ++v) live[v] = (word >> ((ibc + v) & 31)) & 1u;
    }
#pragma unroll
    for (int n0 = 0; n0 < 4 * NT; n0 += NG) {
        float qv[NG][4], rv[NG][4];
#pragma unroll
        for (int n = 0; n < NG; ++n)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t i = i0 + 16 * MT * w + 16 * mt + 4 * g + v;
                const int64_t ic = i < N ? i : N - 1;
                const size_t o = vec_index(N, ldb, ic, (int)(nb0 + 16 * (n0 + n) + c16));
                qv[n][v] = Qs[o];
                const float rr = R[o];
                rv[n][v] = live[v] ? rr : 0.f;
            }
#pragma unroll
        for (int nn = 0; nn < NG; ++nn) {
            const int n = n0 + nn;
            const int col = (int)(nb0 + 16 * n + c16);
            const double av = a[col];
            double ss = 0.0;
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int64_t i = i0 + 16 * MT * w + 16 * mt + 4 * g + v;
                const float q = qv[nn][v] + cc * acc[mt][n][v];
                const float rn = (float)((double)rv[nn][v] - av * (double)q);
                const float r = av != 0.0 ? rn : rv[nn][v];
                if (i < N) R[vec_index(N, ldb, i, col)] = (zmask >> n) & 1u ? 0.f : r;
                ss += i < N ? (double)r * (double)r : 0.0;
            }
            ss += __shfl_xor(ss, 16, kWave);
            ss += __shfl_xor(ss, 32, kWave);
            if (g == 0) sh[MT * w + mt][16 * n + c16] = ss;
        }
    }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < (MT / 2) * 64 * NT; t += kBlock) {
        const int q = t / (64 * NT), c = t % (64 * NT);
        const int64_t grp = rb * (MT / 2) + q;  // 128-row group; ceil(N / 128) of them
        if (grp * 128 >= N) continue;
        double sum = 0.0;
#pragma unroll
        for (int j = 0; j < 8; ++j) sum += sh[8 * q + j][c];
        part[(size_t)grp * ldb + nb0 + c] = sum;
    }
}

int uc_update_r_blocks(int64_t N) { return (int)((N + 127) / 128); }

hipError_t launch_uc_update_r_bf16(int64_t N, UOperand U, int rp, int rk, const unsigned short *CT_hi, const unsigned short *CT_lo, int ldb,
                                   const float *Qs, double alpha, float *R, const double *a, double *part,
                                   IterGuard g, hipStream_t s, int ntr, int width, const uint32_t *rowmask,
                                   const int32_t *iters, const int32_t *maxit) {
    if (rp % 32 != 0 || rk % 32 != 0) return hipErrorInvalidValue;  // whole 32-wide K tiles
    if (iters && (!maxit || rowmask)) return hipErrorInvalidValue;
    if (width == 0) width = ldb;
    if (width % 64 != 0 || width > ldb) return hipErrorInvalidValue;
    const int nt = tn_nt(width, ntr, 2);
    if (nt == 0) return hipErrorInvalidValue;
    const unsigned nblk = (unsigned)(width / (64 * nt)) * (unsigned)((N + 64 * kUcrMt - 1) / (64 * kUcrMt));
    const float cc = (float)(alpha / (1.0 - alpha));
#define HD_UR(AKV, NTV)                                                                                     \
    if (rowmask)                                                                                            \
        k_uc_update_r_tn<AKV, NTV, true><<<nblk, kBlock, 0, s>>>(N, U.hi, U.lo ? U.lo : U.hi, rp, rk, CT_hi, \
                                                                 CT_lo, ldb, Qs, cc, R, a, part, width, g,   \
                                                                 rowmask, nullptr, nullptr);                 \
    else                                                                                                    \
        k_uc_update_r_tn<AKV, NTV, false><<<nblk, kBlock, 0, s>>>(N, U.hi, U.lo ? U.lo : U.hi, rp, rk, CT_hi, \
                                                                  CT_lo, ldb, Qs, cc, R, a, part, width, g,   \
                                                                  nullptr, iters, maxit)
#define HD_UR_NT(AKV) \
    if (nt == 4) { HD_UR(AKV, 4); } else if (nt == 2) { HD_UR(AKV, 2); } else { HD_UR(AKV, 1); }
    switch (akind(U)) {
        case AK_FP8: HD_UR_NT(AK_FP8); break;
        case AK_BF16X2: HD_UR_NT(AK_BF16X2); break;
        default: HD_UR_NT(AK_BF16); break;
    }
#undef HD_UR_NT
#undef HD_UR
    return hipGetLastError();
}

// x[b][i] = (U Cs)[i][b] + X[i][b] (b < B): the product as in u_c over the
// ldc >= B columns of CsT; each wave then writes its tile query-major, one
// 16-item m-tile at a time through LDS, so that every query's 16 items go
// out as one 64-byte run. EMIT (one-pass top-K): each x is offered to its
// query's candidate lists instead (a block's RB items lie in one list
// chunk) and x is not written. gate: the launch returns while *gate == 0.
template <int AK, int NT, bool EMIT, bool FOLD>
__global__ __launch_bounds__(kBlock, 2) void k_combine_tn(int64_t N, int B, const void *__restrict__ U,
                                                       const void *__restrict__ Ul, int rp,
                                                       int rk, const unsigned short *__restrict__ CT_hi,
                                                       const unsigned short *__restrict__ CT_lo, int ldc,
                                                       const float *__restrict__ X, float *__restrict__ x,
                                                       int64_t ldx, TopkLists tl,
                                                       const int32_t *__restrict__ gate, XFold fold) {
    if (!EMIT && gate && *gate == 0) return;
    // FOLD: the guard decides whether the last update applies (a = 0: not)
    const bool fo = FOLD && !all_stopped(fold.g.nact, fold.g.ntile);
    __shared__ float T[4][64][17];
    constexpr int MT = tn_mt(NT), RB = tn_rows(NT);
    const unsigned L = xcd_tile(), ncg = (unsigned)ldc / (64 * NT);
    const int64_t i0 = (int64_t)(L / ncg) * RB;
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    const int64_t nb0 = (int64_t)(L % ncg) * 64 * NT;
    __shared__ EmitStage es;
    __shared__ uint32_t thr[64 * NT];
    if (EMIT) {
        // published by the first barrier of the block GEMM
        for (int t = threadIdx.x; t < 64 * NT; t += kBlock)
            thr[t] = nb0 + t < B ? tl.thr[nb0 + t] : 0u;
        if (threadIdx.x == 0) es.n = 0;
    }
    f32x4 acc[MT][4 * NT];
    tn_block<AK, NT>(U, Ul, rp / 32, i0, N, CT_hi, CT_lo, rk / 32, nb0, 0, rk, acc);
    const int g = lane / 16, c16 = lane % 16;
    // per m-tile (16 items) and group of four n-tiles (64 queries); the
    // m-tile's loads of X (and with FOLD of P) are all issued first
    // (branch-free: rows past N read row N - 1), not one group at a time
    // between the barriers
    // groups of n-tile groups whose P loads are in flight together (with
    // four n-tile groups one at a time, to stay within the registers)
    constexpr int GB = FOLD && NT == 4 ? 1 : NT;
#pragma unroll
    for (int mt = 0; mt < MT; ++mt) {
        const int64_t ib = i0 + 16 * MT * w + 16 * mt;
        float xv[NT][4][4];
#pragma unroll
        for (int n0 = 0; n0 < NT; n0 += GB) {
            float pv[GB][4][4];
#pragma unroll
            for (int ng = n0; ng < n0 + GB; ++ng)
#pragma unroll
                for (int v = 0; v < 4; ++v) {
                    const int64_t i = ib + 4 * g + v;
                    const int64_t ic = i < N ? i : N - 1;
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const size_t o = vec_index(N, ldc, ic, (int)(nb0 + 64 * ng + 16 * q + c16));
                        xv[ng][v][q] = X[o];
                        if (FOLD) pv[ng - n0][v][q] = fold.P[o];
                    }
                }
            if (FOLD) {
#pragma unroll
                for (int ng = n0; ng < n0 + GB; ++ng)
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        const double a = fo ? fold.a[nb0 + 64 * ng + 16 * q + c16] : 0.0;
#pragma unroll
                        for (int v = 0; v < 4; ++v) xv[ng][v][q] = fold_x(xv[ng][v][q], pv[ng - n0][v][q], a);
                    }
            }
        }
#pragma unroll
        for (int ng = 0; ng < NT; ++ng) {
            __syncthreads();
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int rl = 4 * g + v;
#pragma unroll
                for (int q = 0; q < 4; ++q) T[w][16 * q + c16][rl] = acc[mt][4 * ng + q][v] + xv[ng][v][q];
            }
            __syncthreads();
            // lane -> (query bl = f / 16, item f % 16)
            for (int f = lane; f < 64 * 16; f += kWave) {
                const int bl = f / 16, rl = f % 16;
                const int64_t b = nb0 + 64 * ng + bl, i = ib + rl;
                if (b < B && i < N) {
                    if (EMIT)
                        emit_one(es, thr[64 * ng + bl], (int)b, i, T[w][bl][rl]);
                    else
                        x[(size_t)b * ldx + i] = T[w][bl][rl];
                }
            }
        }
    }
    if (EMIT) {
        __syncthreads();
        const int64_t bh = nb0 + 64 * NT < B ? nb0 + 64 * NT : B;
        emit_flush(es, tl, (int)(i0 / kTopkChunk), (int)nb0, (int)bh);
    }
}

int combine_nt(int ldb, int req) { return tn_nt(ldb, req, 2); }

hipError_t launch_combine_bf16(int64_t N, int B, UOperand U, int rp, int rk, const unsigned short *CT_hi,
                               const unsigned short *CT_lo, int ldb, const float *X, float *x,
                               int64_t ldx, hipStream_t s, int ntr, const TopkLists *tl,
                               const int32_t *gate, const XFold *fold) {
    if (rp % 32 != 0 || rk % 32 != 0) return hipErrorInvalidValue;  // whole 32-wide K tiles
    if (tl && (gate || kTopkChunk % tn_rows(1) != 0 || kTopkChunk % tn_rows(4) != 0)) return hipErrorInvalidValue;
    const int nt = tn_nt(ldb, ntr, 2);
    if (nt == 0 || (fold && nt == 4)) return hipErrorInvalidValue;
    const unsigned nblk = (unsigned)(ldb / (64 * nt)) * (unsigned)((N + tn_rows_rt(nt) - 1) / tn_rows_rt(nt));
    const TopkLists none{nullptr, nullptr, nullptr, 0};
    const TopkLists &l = tl ? *tl : none;
    const XFold nofold{nullptr, nullptr, IterGuard{nullptr, 0}};
    const XFold &f = fold ? *fold : nofold;
#define HD_CB2(AKV, NTV, EM, FO)                                                                                \
    k_combine_tn<AKV, NTV, EM, FO><<<nblk, kBlock, 0, s>>>(N, B, U.hi, U.lo ? U.lo : U.hi, rp, rk, CT_hi, CT_lo, ldb, \
                                                           X, x, ldx, l, gate, f)
#define HD_CB(AKV, NTV)                                     \
    do {                                                    \
        if (tl) {                                           \
            if (fold) HD_CB2(AKV, NTV, true, true);         \
            else HD_CB2(AKV, NTV, true, false);             \
        } else {                                            \
            if (fold) HD_CB2(AKV, NTV, false, true);        \
            else HD_CB2(AKV, NTV, false, false);            \
        }                                                   \
    } while (0)
// four n-tiles per wave have no registers left for the fold's P (see
// combine_nt); their callers keep the separate last update
#define HD_CB4(AKV)                                 \
    do {                                            \
        if (tl) HD_CB2(AKV, 4, true, false);        \
        else HD_CB2(AKV, 4, false, false);          \
    } while (0)
#define HD_CB_NT(AKV) \
    if (nt == 4) HD_CB4(AKV); else if (nt == 2) HD_CB(AKV, 2); else HD_CB(AKV, 1)
    switch (akind(U)) {
        case AK_FP8: HD_CB_NT(AK_FP8); break;
        case AK_BF16X2: HD_CB_NT(AK_BF16X2); break;
        default: HD_CB_NT(AK_BF16); break;
    }
#undef HD_CB_NT
#undef HD_CB4
#undef HD_CB
#undef HD_CB2
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Query descriptors split once per batch: Qh / Ql (B64 x ldv bfloat16, B64 =
// B rounded up to 64, in fragment order, zero padded), the hi and lo parts
// of q.
__global__ __launch_bounds__(kBlock) void k_split_q(int B, int B64, int d, int ldv,
                                                    const float *__restrict__ q,
                                                    unsigned short *__restrict__ Qh,
                                                    unsigned short *__restrict__ Ql) {
    const size_t idx = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (idx >= (size_t)B64 * ldv) return;
    // idx runs over the output in fragment order (kt = ldv / 32)
    const int kt = ldv / 32, l = (int)((idx / 8) % 64);
    const size_t tile = idx / 512;
    const int b = (int)(tile / kt) * 16 + l % 16, t = (int)(tile % kt) * 32 + 8 * (l / 16) + (int)(idx % 8);
    const float v = b < B && t < d ? q[(size_t)b * d + t] : 0.f;
    const unsigned short h = bf16_rne(v);
    Qh[idx] = h;
    Ql[idx] = bf16_rne(v - bf16_to_f(h));
}

// sim[b][j] = q[b] . V[j] with V stored bfloat16 (N x ldv in fragment order,
// rows padded to a multiple of 16) and q split hi/lo.
// M = b, N = j, K = t. A block covers 64 queries x 256 items; wave w owns
// items [64w, 64w+64) (four n-tiles) for all 64 queries (four m-tiles, hi
// and lo), so each V fragment feeds eight MFMAs. V rows are read by one wave
// only: each wave loads its V fragments straight from global memory into
// registers, one 32-wide k chunk ahead. The Q tiles (64 x 32, hi and lo:
// eight fragment tiles) are shared by the four waves and staged in LDS per
// chunk in fragment order, so the waves' fragment reads are conflict-free.
// The logical tiles run
// over the query tiles fastest, so the tiles of one item range run on one
// XCD and share V through its L2.
// EMIT (one-pass top-k): every similarity is offered to its query's
// candidate lists (tl) and sim is not written; a block's 256 items lie in
// one list chunk. gate: the whole launch returns while *gate == 0.
template <int VK, bool EMIT>
__global__ __launch_bounds__(kBlock, 3) void k_sim_bf16(int64_t N, int B, int ldv,
                                                     const unsigned short *__restrict__ Qh,
                                                     const unsigned short *__restrict__ Ql,
                                                     const void *__restrict__ V,
                                                     const float *__restrict__ vscale,
                                                     float *__restrict__ sim, int64_t lds, TopkLists tl,
                                                     const int32_t *__restrict__ gate) {
    if (!EMIT && gate && *gate == 0) return;
    __shared__ __attribute__((aligned(16))) unsigned short Qs[2][4][512];
    const int lane = threadIdx.x % kWave, w = threadIdx.x / kWave;
    const int g = lane / 16, c16 = lane % 16;
    const unsigned L = xcd_tile(), nqt = (unsigned)(B + 63) / 64;
    const int b0 = (int)(L % nqt) * 64;
    const int64_t jb = (int64_t)(L / nqt) * 256;
    __shared__ EmitStage es;
    __shared__ uint32_t thr[64];
    if (EMIT) {
        // published by the first barrier of the k loop
        if (threadIdx.x < 64) thr[threadIdx.x] = b0 + (int)threadIdx.x < B ? tl.thr[b0 + threadIdx.x] : 0u;
        if (threadIdx.x == 0) es.n = 0;
    }
    f32x4 acc[4][4];
#pragma unroll
    for (int m = 0; m < 4; ++m)
#pragma unroll
        for (int n = 0; n < 4; ++n) acc[m][n] = f32x4{0.f, 0.f, 0.f, 0.f};
    // this lane's place in its V tiles (one 16-item tile row per n-tile;
    // k chunk t is tile t / 32 of the row, 512 elements on). Loads are
    // unconditional and in bounds (tiles past the last item tile read tile
    // jb / 16, queries past B read row b0, a chunk past ldv reloads the last;
    // none of those results is stored), so the compiler's wait counts stay
    // exact.
    size_t pv[4];  // element offsets (bytes for fp8 codes)
    const int64_t jtiles = (N + 15) / 16;
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const int64_t tb = jb / 16 + 4 * w + n;
        pv[n] = ((size_t)(tb < jtiles ? tb : jb / 16) * (size_t)(ldv / 32) * 64 + (size_t)lane) * 8;
    }
    // Q staging: threads t < 128 copy the hi tiles, the others the lo tiles;
    // thread t copies lane `lane` of m-tiles qm and qm + 2 (qm = (t % 128) /
    // 64). Rows past B are the zero padding of the split.
    const int qa = threadIdx.x / 128, qm = (threadIdx.x % 128) / 64;
    const unsigned short *qsrc =
        (qa == 0 ? Qh : Ql) + ((size_t)(b0 / 16 + qm) * (size_t)(ldv / 32) * 64 + (size_t)lane) * 8;
    const size_t qstep = (size_t)2 * (size_t)(ldv / 32) * 512;  // two tile rows on
    bf16x8 vf[2][4], qv[2];
    auto fetch_v = [&](int slot, int t0) {
        const int tc = t0 < ldv ? t0 : ldv - 32;
#pragma unroll
        for (int n = 0; n < 4; ++n) vf[slot][n] = load_a8<VK>(V, pv[n] + (size_t)tc * 16);
    };
    auto fetch_q = [&](int t0) {
        const int tc = t0 < ldv ? t0 : ldv - 32;
#pragma unroll
        for (int u = 0; u < 2; ++u) qv[u] = load8(qsrc + u * qstep + (size_t)tc * 16);
    };
    fetch_v(0, 0);
    fetch_q(0);
    // two k chunks per trip so that the V register slots have fixed names
    for (int t0 = 0; t0 < ldv; t0 += 64) {
#pragma unroll
        for (int st = 0; st < 2; ++st) {
            const int tt = t0 + 32 * st;
            if (tt < ldv) {
                __syncthreads();
#pragma unroll
                for (int u = 0; u < 2; ++u) *reinterpret_cast<bf16x8 *>(&Qs[qa][qm + 2 * u][8 * lane]) = qv[u];
                __syncthreads();
                fetch_q(tt + 32);
                fetch_v(st ^ 1, tt + 32);
#pragma unroll
                for (int m = 0; m < 4; ++m) {
                    const bf16x8 h = load8(&Qs[0][m][8 * lane]);
                    const bf16x8 l = load8(&Qs[1][m][8 * lane]);
#pragma unroll
                    for (int n = 0; n < 4; ++n) {
                        acc[m][n] = mfma16bf(h, vf[st][n], acc[m][n]);
                        acc[m][n] = mfma16bf(l, vf[st][n], acc[m][n]);
                    }
                }
            }
        }
    }
#pragma unroll
    for (int n = 0; n < 4; ++n) {
        const int64_t j = jb + 64 * w + 16 * n + c16;
        if (j >= N) continue;
        // fp8 descriptors: row j's scale (its codes' products are acc)
        const float sc = VK == AK_FP8 ? vscale[j] : 1.0f;
#pragma unroll
        for (int m = 0; m < 4; ++m)
#pragma unroll
            for (int v = 0; v < 4; ++v) {
                const int bl = 16 * m + 4 * g + v, b = b0 + bl;
                if (b >= B) continue;
                const float val = VK == AK_FP8 ? acc[m][n][v] * sc : acc[m][n][v];
                if (EMIT)
                    emit_one(es, thr[bl], b, j, val);
                else
                    sim[(size_t)b * lds + j] = val;
            }
    }
    if (EMIT) {
        __syncthreads();
        emit_flush(es, tl, (int)(jb / kTopkChunk), b0, b0 + 64 < B ? b0 + 64 : B);
    }
}

hipError_t launch_sim_bf16(int64_t N, int B, int d, const float *q, const void *V,
                           int ldv, unsigned short *qsplit, float *sim, int64_t lds, hipStream_t s,
                           const float *vscale, const TopkLists *tl, const int32_t *gate, bool split_q) {
    if (ldv % 32 != 0) return hipErrorInvalidValue;
    if (tl && (gate || kTopkChunk % 256 != 0)) return hipErrorInvalidValue;
    const int B64 = sim_qsplit_rows(B);
    unsigned short *Qh = qsplit, *Ql = qsplit + (size_t)B64 * ldv;
    const size_t tot = (size_t)B64 * ldv;
    if (split_q) {
        k_split_q<<<(unsigned)((tot + kBlock - 1) / kBlock), kBlock, 0, s>>>(B, B64, d, ldv, q, Qh, Ql);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const unsigned nblk = (unsigned)((B + 63) / 64) * (unsigned)((N + 255) / 256);
    const TopkLists none{nullptr, nullptr, nullptr, 0};
    const TopkLists &l = tl ? *tl : none;
#define HD_SIM(VKV, EM) k_sim_bf16<VKV, EM><<<nblk, kBlock, 0, s>>>(N, B, ldv, Qh, Ql, V, vscale, sim, lds, l, gate)
    if (vscale) {
        if (tl) HD_SIM(AK_FP8, true); else HD_SIM(AK_FP8, false);
    } else {
        if (tl) HD_SIM(AK_BF16, true); else HD_SIM(AK_BF16, false);
    }
#undef HD_SIM
    return hipGetLastError();
}

}  // namespace hd
