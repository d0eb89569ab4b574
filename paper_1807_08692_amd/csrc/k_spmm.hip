// Sparse product with the normalised graph over many right-hand sides, the
// S z part of the operator of Section 4.2, eq. (box):
//     Q = (Zs - alpha * S P) / (1 - alpha),
// where Zs = P + alpha U1 L1 U1^T P (from k_ugemm.hip) or Zs = P when r = 0
// (plain temporal filtering, eq. (temporal)). It also returns per-block
// partials of gamma = P^T Q in double precision.
//
// gfx950 mapping: one wavefront per graph row; the 64 lanes (x CPL columns
// per lane) cover a tile of query columns, so the gathered row P[j, :] of
// each neighbour is one contiguous, fully coalesced load. The wave fetches
// 64 (column id, value) pairs of its row at a time and broadcasts each pair
// with readlane, keeping up to 16 gathers in flight. The kernel is bound by
// HBM (or Infinity Cache) bandwidth: it reads the CSR once, gathers P, and
// streams Zs in and Q out. In the first CG iteration P = y is nonzero on the
// k_y rows of each query only: with the row mask the y scatter builds, that
// product skips the gathers (and, when Zs = P, the own-row loads) of the
// all-zero rows, with a bit-identical result.
//
// Source bands: on this chip a gathered row of P is served from HBM or from
// the 256 MB Infinity Cache, and P (N x ldb fp32) is far larger than that
// cache at a million items. Splitting each row's neighbours into G bands by
// neighbour id (the CSR columns are increasing, so a band is a contiguous
// run of the row, located by the per-row cut offsets built at load time)
// and running one launch per band keeps the rows of P that all waves gather
// at one time to about 1/G of P. A band launch continues each row's fp32
// sum from the partial sum the previous band launch stored in Q, adding its
// edges in the same order as the single pass, so every band count gives
// bit-identical results; only the last band launch applies the operator's
// epilogue and the gamma partials.
#include "hd_device.h"
#include "hd_kernels.h"

namespace hd {

template <int CPL>
struct VecF;
template <>
struct VecF<1> {
    float v[1];
    __device__ __forceinline__ void load(const float *p) { v[0] = *p; }
    __device__ __forceinline__ void store(float *p) const { *p = v[0]; }
};
template <>
struct VecF<2> {
    float v[2];
    __device__ __forceinline__ void load(const float *p) {
        float2 t = *reinterpret_cast<const float2 *>(p);
        v[0] = t.x;
        v[1] = t.y;
    }
    __device__ __forceinline__ void store(float *p) const {
        *reinterpret_cast<float2 *>(p) = make_float2(v[0], v[1]);
    }
};
template <>
struct VecF<4> {
    float v[4];
    __device__ __forceinline__ void load(const float *p) {
        float4 t = *reinterpret_cast<const float4 *>(p);
        v[0] = t.x;
        v[1] = t.y;
        v[2] = t.z;
        v[3] = t.w;
    }
    __device__ __forceinline__ void store(float *p) const {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    }
};

// MASKED: rowmask has bit j set for every row j of P that may be nonzero (the
// support of y in the first CG iteration, where P = y); a neighbour whose bit
// is clear is skipped instead of gathered. Its term would add v * 0 to the
// accumulator, which leaves it unchanged, and the kept terms are added in the
// same order, so the result is bit-identical to the full product.
//
// BANDED: only the row's edges in band [blo, bhi) (in eighths of the id
// range; cut[8 i + b - 1] = the number of row i's edges whose neighbour id
// is below b N / 8) are added; unless `first`, each row's sum starts from
// the partial stored in Q; unless `last`, the sum is stored back to Q and
// nothing else is written.
template <int CPL, bool MASKED, bool BANDED>
__global__ __launch_bounds__(kBlock) void k_spmm(int64_t N, const int64_t *__restrict__ rowptr,
                                                 const int32_t *__restrict__ col,
                                                 const float *__restrict__ val,
                                                 const float *__restrict__ P,
                                                 const float *__restrict__ Zs,
                                                 float *__restrict__ Q, int ldb, float alpha,
                                                 float one_minus_alpha, int64_t rb,
                                                 double *__restrict__ gpart, IterGuard ig,
                                                 const uint32_t *__restrict__ rowmask,
                                                 const int32_t *__restrict__ cut, int blo, int bhi,
                                                 int first, int last) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    const int lane = threadIdx.x % kWave;
    const int w = threadIdx.x / kWave;
    const int c0 = blockIdx.y * (kWave * CPL) + lane * CPL;
    const int64_t rs = (int64_t)blockIdx.x * rb;
    const int64_t re = rs + rb < N ? rs + rb : N;
    double g[CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) g[c] = 0.0;

    for (int64_t i = rs + w; i < re; i += 4) {
        int64_t e0 = rowptr[i], e1 = rowptr[i + 1];
        float acc[CPL];
#pragma unroll
        for (int c = 0; c < CPL; ++c) acc[c] = 0.f;
        if (BANDED) {
            const int32_t *cr = cut + (size_t)i * 8;
            e1 = e0 + cr[bhi - 1];
            e0 += blo > 0 ? cr[blo - 1] : 0;
            if (!first) {
                VecF<CPL> t;
                t.load(Q + (size_t)i * ldb + c0);
#pragma unroll
                for (int c = 0; c < CPL; ++c) acc[c] = t.v[c];
            }
        }
        for (int64_t eb = e0; eb < e1; eb += kWave) {
            const int64_t me = eb + lane;
            int cidx = 0;
            float cv = 0.f;
            if (me < e1) {
                cidx = col[me];
                cv = val[me];
            }
            if (MASKED) {
                // the lanes whose neighbour row is in the mask, in edge order
                const bool nz = me < e1 && ((rowmask[cidx >> 5] >> (cidx & 31)) & 1u);
                uint64_t bits = __ballot(nz);
                while (bits) {
                    const int t = __builtin_ctzll(bits);
                    bits &= bits - 1;
                    const int j = bcast_i(cidx, t);
                    const float v = bcast_f(cv, t);
                    VecF<CPL> pv;
                    pv.load(P + (size_t)j * ldb + c0);
#pragma unroll
                    for (int c = 0; c < CPL; ++c) acc[c] += v * pv.v[c];
                }
                continue;
            }
            const int cnt = (int)(e1 - eb < kWave ? e1 - eb : kWave);
            int t = 0;
            for (; t + 16 <= cnt; t += 16) {
                VecF<CPL> pv[16];
                float vv[16];
#pragma unroll
                for (int u = 0; u < 16; ++u) {
                    const int j = bcast_i(cidx, t + u);
                    vv[u] = bcast_f(cv, t + u);
                    pv[u].load(P + (size_t)j * ldb + c0);
                }
#pragma unroll
                for (int u = 0; u < 16; ++u)
#pragma unroll
                    for (int c = 0; c < CPL; ++c) acc[c] += vv[u] * pv[u].v[c];
            }
            for (; t + 4 <= cnt; t += 4) {
                VecF<CPL> pv[4];
                float vv[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const int j = bcast_i(cidx, t + u);
                    vv[u] = bcast_f(cv, t + u);
                    pv[u].load(P + (size_t)j * ldb + c0);
                }
#pragma unroll
                for (int u = 0; u < 4; ++u)
#pragma unroll
                    for (int c = 0; c < CPL; ++c) acc[c] += vv[u] * pv[u].v[c];
            }
            for (; t < cnt; ++t) {
                const int j = bcast_i(cidx, t);
                const float v = bcast_f(cv, t);
                VecF<CPL> pv;
                pv.load(P + (size_t)j * ldb + c0);
#pragma unroll
                for (int c = 0; c < CPL; ++c) acc[c] += v * pv.v[c];
            }
        }
        if (BANDED && !last) {
            VecF<CPL> t;
#pragma unroll
            for (int c = 0; c < CPL; ++c) t.v[c] = acc[c];
            t.store(Q + (size_t)i * ldb + c0);
            continue;
        }
        VecF<CPL> z, p, q;
        if (MASKED && Zs == P && !((rowmask[i >> 5] >> (i & 31)) & 1u)) {
            // a row outside the mask is zero in P (= Zs here)
#pragma unroll
            for (int c = 0; c < CPL; ++c) z.v[c] = 0.f;
        } else {
            z.load(Zs + (size_t)i * ldb + c0);
        }
        if (Zs == P) {
            p = z;
        } else {
            p.load(P + (size_t)i * ldb + c0);
        }
#pragma unroll
        for (int c = 0; c < CPL; ++c) {
            q.v[c] = (z.v[c] - alpha * acc[c]) / one_minus_alpha;
            g[c] += (double)p.v[c] * (double)q.v[c];
        }
        q.store(Q + (size_t)i * ldb + c0);
    }

    if (BANDED && !last) return;  // no gamma partials before the last band
    __shared__ double sh[4][kWave * CPL];
#pragma unroll
    for (int c = 0; c < CPL; ++c) sh[w][lane * CPL + c] = g[c];
    __syncthreads();
    for (int t = threadIdx.x; t < kWave * CPL; t += kBlock) {
        double s = ((sh[0][t] + sh[1][t]) + sh[2][t]) + sh[3][t];
        gpart[(size_t)blockIdx.x * ldb + blockIdx.y * (kWave * CPL) + t] = s;
    }
}

bool tile_param_ok(int v, int ldb) { return (v == 1 || v == 2 || v == 4) && ldb % (64 * v) == 0; }

bool band_param_ok(int v) { return v == 1 || v == 2 || v == 4 || v == 8; }

void build_band_cuts(int64_t N, const int64_t *rowptr, const int32_t *col, int32_t *cut) {
    for (int64_t i = 0; i < N; ++i) {
        const int64_t s = rowptr[i], e = rowptr[i + 1];
        int64_t k = s;
        for (int b = 1; b <= 8; ++b) {
            const int64_t bound = (int64_t)b * N / 8;  // ids below it lie in bands 0 .. b-1
            while (k < e && col[k] < bound) ++k;
            cut[(size_t)i * 8 + b - 1] = (int32_t)(k - s);
        }
    }
}

// cpl: query columns per lane (a wave covers 64 cpl columns of a row); the
// default is 2 when it divides the width (measured fastest at 256 columns on a
// million-row graph), else 1; the masked product takes the widest that
// divides the width. width (0 = ldb): only columns [0, width) are
// computed (row stride stays ldb); a multiple of 64. rowmask (nullptr =
// none): bit j of word j / 32 set for the rows of P that may be nonzero;
// the others must be zero in every computed column. bands (0 or 1 = one
// pass; 2, 4, 8 with cut): source bands, one launch each, bit-identical
// results; not combined with rowmask (the masked product gathers few rows).
hipError_t launch_spmm(int64_t N, const int64_t *rowptr, const int32_t *col, const float *val,
                       const float *P, const float *Zs, float *Q, int ldb, double alpha,
                       RowPart rp, double *gpart, IterGuard g, hipStream_t s, int cpl, int width,
                       const uint32_t *rowmask, int bands, const int32_t *cut) {
    const float a = (float)alpha, oma = (float)(1.0 - alpha);
    if (width == 0) width = ldb;
    if (width < 64 || width > ldb || width % 64 != 0) return hipErrorInvalidValue;
    if (cpl == 0) cpl = width % 128 == 0 ? 2 : 1;
    if (!tile_param_ok(cpl, width)) return hipErrorInvalidValue;
    // the masked product is bound by each row's chain of dependent loads
    // (row pointers, column ids, mask words, the few gathers), which every
    // column slice repeats: one wave covers as many columns as it can
    if (rowmask) cpl = width % 256 == 0 ? 4 : width % 128 == 0 ? 2 : 1;
    if (bands == 0 || rowmask) bands = 1;
    if (!band_param_ok(bands) || (bands > 1 && !cut)) return hipErrorInvalidValue;
    const dim3 grid((unsigned)rp.nblk, (unsigned)(width / (64 * cpl)));
#define HD_SPMM(C, M, BD, LO, HI, FI, LA)                                                                        \
    k_spmm<C, M, BD><<<grid, kBlock, 0, s>>>(N, rowptr, col, val, P, Zs, Q, ldb, a, oma, rp.rb, gpart, g, rowmask, \
                                             cut, LO, HI, FI, LA)
    if (rowmask) {
        if (cpl == 1) HD_SPMM(1, true, false, 0, 8, 1, 1);
        else if (cpl == 2) HD_SPMM(2, true, false, 0, 8, 1, 1);
        else HD_SPMM(4, true, false, 0, 8, 1, 1);
    } else if (bands == 1) {
        if (cpl == 1) HD_SPMM(1, false, false, 0, 8, 1, 1);
        else if (cpl == 2) HD_SPMM(2, false, false, 0, 8, 1, 1);
        else HD_SPMM(4, false, false, 0, 8, 1, 1);
    } else {
        const int step = 8 / bands;
        for (int b = 0; b < bands; ++b) {
            const int lo = b * step, hi = lo + step, fi = b == 0, la = b == bands - 1;
            if (cpl == 1) HD_SPMM(1, false, true, lo, hi, fi, la);
            else if (cpl == 2) HD_SPMM(2, false, true, lo, hi, fi, la);
            else HD_SPMM(4, false, true, lo, hi, fi, la);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
    }
#undef HD_SPMM
    return hipGetLastError();
}

}  // namespace hd
