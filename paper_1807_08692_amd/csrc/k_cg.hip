// Conjugate-gradient vector and scalar kernels for the temporal term
// (Section 4.2, eq. (h-temporal); Section 5: CG from x0 = 0).
//
// B query columns are solved side by side as independent CG recurrences
// (not block CG): every dot product, step size and stopping test is per
// column and in double precision, the vectors are fp32. Per-block partial
// sums are reduced in a fixed order, so a column's result does not depend on
// which other columns share the batch.
//
// One iteration, for each active column c:
//   Q = A P                                   (k_spmm.hip, k_ugemm.hip)
//   gamma = P^T Q ; a = rho / gamma           (cg_step_a)
//   R -= a Q ; rho' = R^T R                   (update_r)
//   stop if sqrt(rho'/rho0) <= tol ; beta = rho'/rho   (cg_step_b)
//   X += a P ; P = R + beta P                 (update_xp)
#include "hd_device.h"
#include "hd_kernels.h"

namespace hd {

enum { COL_CONVERGED = 0, COL_MAXITER = 1, COL_ZERO_RHS = 2, COL_BREAKDOWN = 3 };

RowPart make_row_part(int64_t N) {
    // at most ~2048 blocks so that the scalar kernels reduce few partials
    int64_t rb = (N + 2047) / 2048;
    rb = ((rb + 63) / 64) * 64;
    if (rb < 64) rb = 64;
    RowPart p;
    p.rb = rb;
    p.nblk = (int)((N + rb - 1) / rb);
    if (p.nblk < 1) p.nblk = 1;
    return p;
}

__global__ __launch_bounds__(kBlock) void k_fill_zero(float4 *p, size_t n4, float *tail, int ntail) {
    size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    size_t stride = (size_t)gridDim.x * kBlock;
    for (; i < n4; i += stride) p[i] = make_float4(0.f, 0.f, 0.f, 0.f);
    if (blockIdx.x == 0 && (int)threadIdx.x < ntail) tail[threadIdx.x] = 0.f;
}

hipError_t launch_fill_zero(float *p, size_t n, hipStream_t s) {
    if (n == 0) return hipSuccess;
    size_t n4 = n / 4;
    int ntail = (int)(n - n4 * 4);
    size_t want = (n4 + kBlock - 1) / kBlock;
    int grid = (int)(want < 8192 ? (want > 0 ? want : 1) : 8192);
    k_fill_zero<<<grid, kBlock, 0, s>>>(reinterpret_cast<float4 *>(p), n4, p + n4 * 4, ntail);
    return hipGetLastError();
}

// Zero every row of R and P that some y of the batch touches (all ldb
// columns): with the first CG iteration reading R and P only on those rows
// (row mask) and writing every row, the scatter of y then needs no full
// fill of R and P. One wave per y row; ids outside [0, N) are skipped (the
// scatter flags them). Rows repeated across y rows are zeroed more than
// once, with the same value.
__global__ __launch_bounds__(kBlock) void k_zero_yrows(int B, int ky, const int32_t *__restrict__ ids, int64_t N,
                                                       int ldb, float *__restrict__ R, float *__restrict__ P) {
    const int lane = threadIdx.x % kWave;
    const int t = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (t >= B) return;  // whole waves
    const int32_t *row = ids + (size_t)t * ky;
    const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
    for (int u = 0; u < ky; ++u) {
        const int32_t id = row[u];
        if (id < 0 || (int64_t)id >= N) continue;
        for (int c = 4 * lane; c < ldb; c += 4 * kWave) {
            const size_t o = vec_index(N, ldb, id, c);
            *reinterpret_cast<float4 *>(R + o) = z;
            *reinterpret_cast<float4 *>(P + o) = z;
        }
    }
}

hipError_t launch_zero_yrows(int B, int ky, const int32_t *ids, int64_t N, int ldb, float *R, float *P,
                             hipStream_t s) {
    if (B <= 0 || ky <= 0) return hipSuccess;
    if (ldb % 4 != 0) return hipErrorInvalidValue;
    const int per = kBlock / kWave;
    k_zero_yrows<<<(B + per - 1) / per, kBlock, 0, s>>>(B, ky, ids, N, ldb, R, P);
    return hipGetLastError();
}

// R, P = y (dense, node-major) from the sparse y of each column; R and P are
// zero in the columns written. One wave per y row: the lane holding the
// first occurrence of an id sums the values of all its occurrences in index
// order and writes the entry (no atomics), so a column's R and P do not
// depend on timing even when an id repeats. Ids outside [0, N) are skipped
// and flagged in *err.
__global__ __launch_bounds__(kBlock) void k_scatter_y(int B, int ky, const int32_t *__restrict__ ids,
                                                      const float *__restrict__ vals, int64_t N, int ldb,
                                                      float *__restrict__ R, float *__restrict__ P,
                                                      int32_t *err, const int32_t *__restrict__ colmap,
                                                      uint32_t *rowmask) {
    const int lane = threadIdx.x % kWave;
    const int t = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (t >= B) return;  // whole waves
    const int b = colmap ? colmap[t] : t;
    const int32_t *row = ids + (size_t)t * ky;
    const float *rv = vals + (size_t)t * ky;
    for (int u = lane; u < ky; u += kWave) {
        const int32_t id = row[u];
        if (id < 0 || (int64_t)id >= N) {
            atomicOr(err, 1);
            continue;
        }
        bool first = true;
        for (int v = 0; v < u && first; ++v) first = row[v] != id;
        if (!first) continue;
        float acc = rv[u];
        for (int v = u + 1; v < ky; ++v)
            if (row[v] == id) acc += rv[v];
        const size_t o = vec_index(N, ldb, id, b);
        R[o] = acc;
        P[o] = acc;
        if (rowmask) atomicOr(&rowmask[id >> 5], 1u << (id & 31));
    }
}

hipError_t launch_scatter_y(int B, int ky, const int32_t *ids, const float *vals, int64_t N,
                            int ldb, float *R, float *P, int32_t *err, hipStream_t s,
                            const int32_t *colmap, uint32_t *rowmask) {
    if (B <= 0 || ky <= 0) return hipSuccess;
    const int per = kBlock / kWave;
    k_scatter_y<<<(B + per - 1) / per, kBlock, 0, s>>>(B, ky, ids, vals, N, ldb, R, P, err, colmap, rowmask);
    return hipGetLastError();
}

// Each thread owns 4 consecutive columns (one float4) of one row; the
// kBlock/G threads of a block that own the same columns step over the
// block's rows together, then combine in LDS in a fixed order.
__device__ __forceinline__ void block_colsum4(double s0, double s1, double s2, double s3, int G,
                                              double *out /* ldb-strided row of partials */) {
    __shared__ double sh[kBlock * 4];
    int t = threadIdx.x;
    sh[t * 4 + 0] = s0;
    sh[t * 4 + 1] = s1;
    sh[t * 4 + 2] = s2;
    sh[t * 4 + 3] = s3;
    __syncthreads();
    int rows = kBlock / G;
    if (t < G) {
        double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
        for (int rr = 0; rr < rows; ++rr) {
            const double *q = sh + (rr * G + t) * 4;
            a0 += q[0];
            a1 += q[1];
            a2 += q[2];
            a3 += q[3];
        }
        out[t * 4 + 0] = a0;
        out[t * 4 + 1] = a1;
        out[t * 4 + 2] = a2;
        out[t * 4 + 3] = a3;
    }
}

// rho0 = y^T y per column straight from y: R holds y after the scatter and
// is zero elsewhere, so the column sum of R^2 over all rows is the sum over
// the distinct ids of the column's y (duplicate ids were added into one
// entry). One wave per y row t (column colmap[t], or t): lane u squares the
// entry of id u unless an earlier id repeats it, and the wave sums 64 ids at
// a time in a fixed order (lane 0's butterfly), so the result depends on the
// ids alone. Without colmap, columns B .. ldb-1 get 0.
__global__ __launch_bounds__(kBlock) void k_ynorm_part(int B, int ky, const int32_t *__restrict__ ids,
                                                       int64_t N, int ldb, const float *__restrict__ R,
                                                       double *__restrict__ part,
                                                       const int32_t *__restrict__ colmap) {
    const int lane = threadIdx.x % kWave;
    const int t = blockIdx.x * (kBlock / kWave) + threadIdx.x / kWave;
    if (t >= (colmap ? B : ldb)) return;  // whole waves
    if (t >= B) {
        if (lane == 0) part[t] = 0.0;
        return;
    }
    const int col = colmap ? colmap[t] : t;
    const int32_t *row = ids + (size_t)t * ky;
    double sum = 0.0;
    for (int u0 = 0; u0 < ky; u0 += kWave) {
        const int u = u0 + lane;
        double x2 = 0.0;
        if (u < ky) {
            const int32_t id = row[u];
            if (id >= 0 && (int64_t)id < N) {
                bool dup = false;
                for (int v = 0; v < u && !dup; ++v) dup = row[v] == id;
                if (!dup) {
                    const double x = (double)R[vec_index(N, ldb, id, col)];
                    x2 = x * x;
                }
            }
        }
        for (int off = kWave / 2; off > 0; off >>= 1) x2 += __shfl_xor(x2, off, kWave);
        sum += x2;
    }
    if (lane == 0) part[col] = sum;
}

hipError_t launch_ynorm_part(int B, int ky, const int32_t *ids, int64_t N, int ldb, const float *R,
                             double *part, hipStream_t s, const int32_t *colmap) {
    const int waves = colmap ? B : ldb;
    if (waves <= 0) return hipSuccess;
    const int per = kBlock / kWave;
    k_ynorm_part<<<(waves + per - 1) / per, kBlock, 0, s>>>(B, ky, ids, N, ldb, R, part, colmap);
    return hipGetLastError();
}

// Fixed-order reduction of nblk per-block partials for the 64 columns of this
// block's tile. The scalar kernels run 1024 threads (16 waves) per tile:
// wave w sums partial rows w, w+16, w+32, ... with four independent
// accumulators (so many loads are in flight), then the 16 wave sums are added
// in order. The order depends on nblk only, never on timing.
constexpr int kScalarThreads = 1024;
constexpr int kScalarWaves = kScalarThreads / kWave;

__device__ __forceinline__ double tile_reduce(const double *part, int nblk, int ldb, int col) {
    __shared__ double sh[kScalarWaves][kWave];
    const int w = threadIdx.x / kWave, lane = threadIdx.x % kWave;
    double a0 = 0, a1 = 0, a2 = 0, a3 = 0;
    int g = w;
    for (; g + 3 * kScalarWaves < nblk; g += 4 * kScalarWaves) {
        a0 += part[(size_t)g * ldb + col];
        a1 += part[(size_t)(g + kScalarWaves) * ldb + col];
        a2 += part[(size_t)(g + 2 * kScalarWaves) * ldb + col];
        a3 += part[(size_t)(g + 3 * kScalarWaves) * ldb + col];
    }
    for (; g < nblk; g += kScalarWaves) a0 += part[(size_t)g * ldb + col];
    sh[w][lane] = (a0 + a1) + (a2 + a3);
    __syncthreads();
    double t = 0.0;
    for (int v = 0; v < kScalarWaves; ++v) t += sh[v][lane];
    return t;
}

__global__ __launch_bounds__(kScalarThreads) void k_cg_init(int B, int ldb, const double *part, int nblk,
                                                    CgState st) {
    int lane = threadIdx.x % kWave;
    int c = blockIdx.x * kWave + lane;
    double rho0 = tile_reduce(part, nblk, ldb, c);
    __shared__ int cnt[kWave];
    if (threadIdx.x < kWave) {
        int act = 0, stat;
        if (c >= B || rho0 == 0.0) {
            stat = COL_ZERO_RHS;
            rho0 = 0.0;
        } else if (!(rho0 > 0.0) || !isfinite(rho0)) {
            stat = COL_BREAKDOWN;
        } else {
            stat = COL_MAXITER;
            act = 1;
        }
        st.rho0[c] = rho0;
        st.rho[c] = rho0;
        st.a[c] = 0.0;
        st.beta[c] = 0.0;
        st.relres[c] = 0.0;
        st.active[c] = act;
        st.iters[c] = 0;
        st.status[c] = stat;
        cnt[lane] = act;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int n = 0;
        for (int l = 0; l < kWave; ++l) n += cnt[l];
        st.nact_part[blockIdx.x] = n;
    }
}

hipError_t launch_cg_init(int B, int ldb, const double *part, int nblk, CgState st, hipStream_t s) {
    k_cg_init<<<ldb / kWave, kScalarThreads, 0, s>>>(B, ldb, part, nblk, st);
    return hipGetLastError();
}

// Partial-sum rows pre-reduced in parallel for the scalar kernels below: a
// tile's 1024 threads reading thousands of rows alone are latency-bound
// (about 50 us for 7,800 rows of 256 columns). Block (tile, s) sums rows
// [s per, (s + 1) per) of its 64 columns, per = ceil(nblk / kPreSplit), in
// tile_reduce's order and writes row s of out; the scalar kernel then sums
// the kPreSplit rows. The order depends on nblk only.
constexpr int kPreSplit = kPreSplitRows;
__global__ __launch_bounds__(kScalarThreads) void k_part_prereduce(const double *part, int nblk, int ldb,
                                                                   double *out, IterGuard ig) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    const int lane = threadIdx.x % kWave;
    const int c = blockIdx.x * kWave + lane;
    const int per = (nblk + kPreSplit - 1) / kPreSplit;
    const int lo = blockIdx.y * per;
    const int hi = lo + per < nblk ? lo + per : nblk;
    const double t = tile_reduce(part + (size_t)(lo < nblk ? lo : 0) * ldb, hi > lo ? hi - lo : 0, ldb, c);
    if (threadIdx.x < kWave) out[(size_t)blockIdx.y * ldb + c] = t;
}

// With scratch (kPreSplit rows of ldb doubles) and more than 2 kPreSplit
// rows, pre-reduce part into scratch; returns the rows the scalar kernel
// then reads (and how many) through *rows / *n.
static hipError_t prereduce(const double *part, int nblk, int ldb, double *scratch, IterGuard g, hipStream_t s,
                            const double **rows, int *n) {
    *rows = part;
    *n = nblk;
    if (!scratch || nblk <= 2 * kPreSplit) return hipSuccess;
    k_part_prereduce<<<dim3((unsigned)(ldb / kWave), kPreSplit), kScalarThreads, 0, s>>>(part, nblk, ldb, scratch, g);
    *rows = scratch;
    *n = kPreSplit;
    return hipGetLastError();
}

// gamma = P^T Q per column; a = rho / gamma, or stop the column (breakdown)
// when gamma is not positive and finite.
__global__ __launch_bounds__(kScalarThreads) void k_cg_step_a(int ldb, const double *gpart, int nblk,
                                                      CgState st, IterGuard ig, const double *gpart2,
                                                      int nblk2) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    int lane = threadIdx.x % kWave;
    int c = blockIdx.x * kWave + lane;
    double gamma = tile_reduce(gpart, nblk, ldb, c);
    if (gpart2) {
        __syncthreads();  // tile_reduce's LDS is reused
        gamma += tile_reduce(gpart2, nblk2, ldb, c);
    }
    if (threadIdx.x < kWave) {
        double a = 0.0;
        if (st.active[c]) {
            if (!(gamma > 0.0) || !isfinite(gamma)) {
                st.status[c] = COL_BREAKDOWN;
                st.active[c] = 0;
            } else {
                a = st.rho[c] / gamma;
            }
        }
        st.a[c] = a;
    }
}

hipError_t launch_cg_step_a(int ldb, const double *gpart, int nblk, CgState st, IterGuard g,
                            hipStream_t s, const double *gpart2, int nblk2, double *scratch) {
    hipError_t e = prereduce(gpart, nblk, ldb, scratch, g, s, &gpart, &nblk);
    if (e == hipSuccess && gpart2)
        e = prereduce(gpart2, nblk2, ldb, scratch ? scratch + (size_t)kPreSplit * ldb : nullptr, g, s, &gpart2,
                      &nblk2);
    if (e != hipSuccess) return e;
    k_cg_step_a<<<ldb / kWave, kScalarThreads, 0, s>>>(ldb, gpart, nblk, st, g, gpart2, nblk2);
    return hipGetLastError();
}

// R -= a Q, and per-block partials of the new R^T R. rowmask (the first CG
// iteration, when R was zeroed only on the rows of y): rows outside it are
// taken as zero in R and not read.
__global__ __launch_bounds__(kBlock) void k_update_r(int64_t N, int ldb, const float *Q, float *R,
                                                     int64_t rb, const double *a, double *part,
                                                     IterGuard ig, const uint32_t *rowmask) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    const int G = ldb / 4;
    const int rows = kBlock / G;
    int cg = threadIdx.x % G;
    int r0 = threadIdx.x / G;
    double a0 = a[cg * 4 + 0], a1 = a[cg * 4 + 1], a2 = a[cg * 4 + 2], a3 = a[cg * 4 + 3];
    int64_t rs = (int64_t)blockIdx.x * rb;
    int64_t re = rs + rb < N ? rs + rb : N;
    double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
    for (int64_t i = rs + r0; i < re; i += rows) {
        const size_t o = vec_index(N, ldb, i, cg * 4);
        float4 *rp = reinterpret_cast<float4 *>(R + o);
        float4 q = *reinterpret_cast<const float4 *>(Q + o);
        float4 r = row_live(rowmask, (int64_t)i) ? *rp : make_float4(0.f, 0.f, 0.f, 0.f);
        // a = 0 leaves a stopped column untouched even if its Q is not finite
        if (a0 != 0.0) r.x = (float)((double)r.x - a0 * (double)q.x);
        if (a1 != 0.0) r.y = (float)((double)r.y - a1 * (double)q.y);
        if (a2 != 0.0) r.z = (float)((double)r.z - a2 * (double)q.z);
        if (a3 != 0.0) r.w = (float)((double)r.w - a3 * (double)q.w);
        *rp = r;
        s0 += (double)r.x * r.x;
        s1 += (double)r.y * r.y;
        s2 += (double)r.z * r.z;
        s3 += (double)r.w * r.w;
    }
    block_colsum4(s0, s1, s2, s3, G, part + (size_t)blockIdx.x * ldb);
}

hipError_t launch_update_r(int64_t N, int ldb, const float *Q, float *R, RowPart rp,
                           const double *a, double *part, IterGuard g, hipStream_t s,
                           const uint32_t *rowmask) {
    k_update_r<<<rp.nblk, kBlock, 0, s>>>(N, ldb, Q, R, rp.rb, a, part, g, rowmask);
    return hipGetLastError();
}

// rho' = R^T R per column; stopping test sqrt(rho'/rho0) <= tol after the
// update; beta = rho'/rho for the columns that go on.
// part == nullptr: the last of a fixed number of products, whose residual
// is not formed: each active column counts the product and stops (status
// stays MAXITER, rho that of the residual before the product).
__global__ __launch_bounds__(kScalarThreads) void k_cg_step_b(int ldb, const double *part, int nblk,
                                                      double tol, CgState st, IterGuard ig,
                                                      int32_t *nact_out) {
    if (all_stopped(ig.nact, ig.ntile)) {
        // nothing ran: carry the (zero) counts over to the other parity
        if (threadIdx.x == 0) nact_out[blockIdx.x] = 0;
        return;
    }
    int lane = threadIdx.x % kWave;
    int c = blockIdx.x * kWave + lane;
    if (!part) {
        if (threadIdx.x < kWave && st.active[c]) {
            st.iters[c] += 1;
            st.active[c] = 0;
        }
        if (threadIdx.x == 0) nact_out[blockIdx.x] = 0;
        return;
    }
    double rho_new = tile_reduce(part, nblk, ldb, c);
    __shared__ int cnt[kWave];
    if (threadIdx.x < kWave) {
        int act = st.active[c];
        if (act) {
            const int it = st.iters[c] + 1;
            st.iters[c] = it;
            double rel = sqrt(rho_new / st.rho0[c]);
            if (rel <= tol) {
                st.status[c] = COL_CONVERGED;
                st.active[c] = 0;
                act = 0;
            } else {
                st.beta[c] = rho_new / st.rho[c];
                if (st.maxit && it >= st.maxit[c]) {  // per-column cap: status stays MAXITER
                    st.active[c] = 0;
                    act = 0;
                }
            }
            st.rho[c] = rho_new;
        }
        cnt[lane] = act;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        int n = 0;
        for (int l = 0; l < kWave; ++l) n += cnt[l];
        nact_out[blockIdx.x] = n;
    }
}

hipError_t launch_cg_step_b(int ldb, const double *part, int nblk, double tol, CgState st,
                            IterGuard g, int32_t *nact_out, hipStream_t s, double *scratch) {
    const hipError_t e = part ? prereduce(part, nblk, ldb, scratch, g, s, &part, &nblk) : hipSuccess;
    if (e != hipSuccess) return e;
    k_cg_step_b<<<ldb / kWave, kScalarThreads, 0, s>>>(ldb, part, nblk, tol, st, g, nact_out);
    return hipGetLastError();
}

// X += a P (the step of this iteration); P = R + beta P for columns still
// active after the stopping test.
// XONLY: the last iteration's update, x += a p alone (no later iteration
// reads the new p), with the same x arithmetic. rowmask (the first CG
// iteration, when only the rows of y were zeroed): X is taken as zero and
// not read, P as zero outside the mask; every row is written.
template <bool XONLY>
__global__ __launch_bounds__(kBlock) void k_update_xp(int64_t N, int ldb, int width, float *X, float *P,
                                                      const float *R, const double *a,
                                                      const double *beta, const int32_t *active,
                                                      IterGuard ig, const uint32_t *rowmask) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    const int G = width / 4;  // columns [0, width) of rows of stride ldb
    const int rows = kBlock / G;
    int cg = threadIdx.x % G;
    int r0 = threadIdx.x / G;
    double a0 = a[cg * 4 + 0], a1 = a[cg * 4 + 1], a2 = a[cg * 4 + 2], a3 = a[cg * 4 + 3];
    double b0 = beta[cg * 4 + 0], b1 = beta[cg * 4 + 1], b2 = beta[cg * 4 + 2], b3 = beta[cg * 4 + 3];
    int k0 = active[cg * 4 + 0], k1 = active[cg * 4 + 1], k2 = active[cg * 4 + 2], k3 = active[cg * 4 + 3];
    size_t total = (size_t)N;
    for (size_t i = (size_t)blockIdx.x * rows + r0; i < total; i += (size_t)gridDim.x * rows) {
        const size_t o = vec_index(N, ldb, (int64_t)i, cg * 4);
        float4 *xp = reinterpret_cast<float4 *>(X + o);
        float4 *pp = reinterpret_cast<float4 *>(P + o);
        const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
        float4 x = rowmask ? z4 : *xp, p = row_live(rowmask, (int64_t)i) ? *pp : z4;
        if (a0 != 0.0) x.x = (float)((double)x.x + a0 * (double)p.x);
        if (a1 != 0.0) x.y = (float)((double)x.y + a1 * (double)p.y);
        if (a2 != 0.0) x.z = (float)((double)x.z + a2 * (double)p.z);
        if (a3 != 0.0) x.w = (float)((double)x.w + a3 * (double)p.w);
        if (XONLY) {
            *xp = x;
            continue;
        }
        const float4 r = *reinterpret_cast<const float4 *>(R + o);
        if (k0) p.x = (float)((double)r.x + b0 * (double)p.x);
        if (k1) p.y = (float)((double)r.y + b1 * (double)p.y);
        if (k2) p.z = (float)((double)r.z + b2 * (double)p.z);
        if (k3) p.w = (float)((double)r.w + b3 * (double)p.w);
        *xp = x;
        *pp = p;
    }
}

hipError_t launch_update_xp(int64_t N, int ldb, float *X, float *P, const float *R,
                            const double *a, const double *beta, const int32_t *active,
                            IterGuard g, hipStream_t s, int width, bool x_only, const uint32_t *rowmask) {
    if (width == 0) width = ldb;
    if (width % 64 != 0 || width > ldb || width > 4 * kBlock) return hipErrorInvalidValue;
    int rows = kBlock / (width / 4);
    int64_t want = (N + rows - 1) / rows;
    int grid = (int)(want < 16384 ? want : 16384);
    if (grid < 1) grid = 1;
    if (x_only)
        k_update_xp<true><<<grid, kBlock, 0, s>>>(N, ldb, width, X, P, R, a, beta, active, g, rowmask);
    else
        k_update_xp<false><<<grid, kBlock, 0, s>>>(N, ldb, width, X, P, R, a, beta, active, g, rowmask);
    return hipGetLastError();
}

// update_xp for the bfloat16 forms of U1: the same X and P updates, and the
// new P also written as its split transpose PT_hi / PT_lo (ldb x ldpt
// bfloat16 in fragment order over items, zero past N), the operand of the
// next iteration's U1^T P. A block covers 64 items x 64 columns: thread t
// updates the float4 at column 4(t%16) of rows t/16 + 16j, then the 64 x 64
// tile of new P is transposed through LDS and thread t writes column t/4,
// items 16(t%4) .. +15 of PT as two 16-byte lane pieces.
//
// SERVE (a server's running solve, iters = the columns' iteration counts):
// a column's first update (iters 1) overwrites X with a p instead of adding
// to the previous occupant's x, and a stopped column's P is set to zero and
// its nonzero R entries are written back as zero, so a column freed by a
// finished request is clean for its next admission without a pass of its
// own (the rows of X, P and PT are written here anyway, those of R read;
// a column ended by its cap already had its last r stored as zero by the
// residual update, so only those stopped by the tolerance write R here).
template <bool SERVE>
__global__ __launch_bounds__(kBlock) void k_update_xp_pt(int64_t N, int ldb, float *X, float *P,
                                                         float *R, const double *a,
                                                         const double *beta, const int32_t *active,
                                                         int64_t ldpt, unsigned short *PTh,
                                                         unsigned short *PTl, IterGuard ig,
                                                         const uint32_t *rowmask, const int32_t *iters) {
    if (all_stopped(ig.nact, ig.ntile)) return;
    __shared__ float T[64][65];
    const int64_t i0 = (int64_t)blockIdx.x * 64;
    const int b0 = blockIdx.y * 64;
    const int c4 = 4 * (threadIdx.x % 16);
    double av[4], bv[4];
    int kv[4];
    bool fresh[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        av[q] = a[b0 + c4 + q];
        bv[q] = beta[b0 + c4 + q];
        kv[q] = active[b0 + c4 + q];
        fresh[q] = SERVE && iters[b0 + c4 + q] == 1;
    }
    // the four rows' loads first, unconditionally (a row past N reads row
    // N - 1 and stores nothing), so all twelve are in flight together; with
    // rowmask (first iteration) X is zero and P zero outside the mask
    float4 xv[4], pv[4], rv[4];
    const float4 z4 = make_float4(0.f, 0.f, 0.f, 0.f);
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int64_t i = i0 + threadIdx.x / 16 + 16 * j;
        const int64_t ic = i < N ? i : N - 1;
        const size_t o = vec_index(N, ldb, ic, b0 + c4);
        xv[j] = rowmask ? z4 : *reinterpret_cast<const float4 *>(X + o);
        pv[j] = row_live(rowmask, ic) ? *reinterpret_cast<const float4 *>(P + o) : z4;
        rv[j] = *reinterpret_cast<const float4 *>(R + o);
    }
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int r = threadIdx.x / 16 + 16 * j;
        const int64_t i = i0 + r;
        float xs[4] = {xv[j].x, xv[j].y, xv[j].z, xv[j].w}, ps[4] = {pv[j].x, pv[j].y, pv[j].z, pv[j].w};
        float rs[4] = {rv[j].x, rv[j].y, rv[j].z, rv[j].w};
        bool rclear = false;
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            if (av[q] != 0.0) xs[q] = (float)((double)(fresh[q] ? 0.f : xs[q]) + av[q] * (double)ps[q]);
            if (kv[q]) {
                ps[q] = (float)((double)rs[q] + bv[q] * (double)ps[q]);
            } else if (SERVE) {
                ps[q] = 0.f;
                rclear |= rs[q] != 0.f;
                rs[q] = 0.f;
            }
        }
        if (i < N) {
            const size_t o = vec_index(N, ldb, i, b0 + c4);
            *reinterpret_cast<float4 *>(X + o) = make_float4(xs[0], xs[1], xs[2], xs[3]);
            *reinterpret_cast<float4 *>(P + o) = make_float4(ps[0], ps[1], ps[2], ps[3]);
            // an active column's r is written back as it was read
            if (SERVE && rclear) *reinterpret_cast<float4 *>(R + o) = make_float4(rs[0], rs[1], rs[2], rs[3]);
        }
        // items past N stay zero in the transpose
#pragma unroll
        for (int q = 0; q < 4; ++q) T[c4 + q][r] = i < N ? ps[q] : 0.f;
    }
    __syncthreads();
    typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));
    const int b = threadIdx.x / 4, seg = 16 * (threadIdx.x % 4);
    bf16x8_t h[2], l[2];
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
        *reinterpret_cast<bf16x8_t *>(PTh + o) = h[u];
        *reinterpret_cast<bf16x8_t *>(PTl + o) = l[u];
    }
}

hipError_t launch_update_xp_pt(int64_t N, int ldb, float *X, float *P, float *R,
                               const double *a, const double *beta, const int32_t *active,
                               int64_t ldpt, unsigned short *PTh, unsigned short *PTl, IterGuard g,
                               hipStream_t s, const uint32_t *rowmask, int width, const int32_t *iters) {
    if (width == 0) width = ldb;
    if (ldpt % 64 != 0 || ldpt < N || ldb % 64 != 0 || width % 64 != 0 || width > ldb)
        return hipErrorInvalidValue;
    if (iters && rowmask) return hipErrorInvalidValue;
    const dim3 grid((unsigned)(ldpt / 64), (unsigned)(width / 64));
    if (iters)
        k_update_xp_pt<true><<<grid, kBlock, 0, s>>>(N, ldb, X, P, R, a, beta, active, ldpt, PTh, PTl, g, rowmask,
                                                     iters);
    else
        k_update_xp_pt<false><<<grid, kBlock, 0, s>>>(N, ldb, X, P, R, a, beta, active, ldpt, PTh, PTl, g, rowmask,
                                                      nullptr);
    return hipGetLastError();
}

// One step of the polynomial filter's Horner recurrence (Appendix A):
// P = c R + qs Q, with R holding y and Q = S_r P_old / 2 (qs = 2), or
// P = c R when qs = 0 (Q not read).
__global__ __launch_bounds__(kBlock) void k_filter_axpy(size_t n4, float4 *P, const float4 *R,
                                                        const float4 *Q, float c, float qs) {
    const size_t i = (size_t)blockIdx.x * kBlock + threadIdx.x;
    if (i >= n4) return;
    const float4 r = R[i];
    float4 p = make_float4(c * r.x, c * r.y, c * r.z, c * r.w);
    if (qs != 0.f) {
        const float4 q = Q[i];
        p = make_float4(p.x + qs * q.x, p.y + qs * q.y, p.z + qs * q.z, p.w + qs * q.w);
    }
    P[i] = p;
}

hipError_t launch_filter_axpy(float *P, const float *R, const float *Q, size_t n, double c, double qs,
                              hipStream_t s) {
    if (n % 4 != 0) return hipErrorInvalidValue;  // solver widths are multiples of 64
    const size_t n4 = n / 4;
    if (n4 == 0) return hipSuccess;
    k_filter_axpy<<<(unsigned)((n4 + kBlock - 1) / kBlock), kBlock, 0, s>>>(
        n4, reinterpret_cast<float4 *>(P), reinterpret_cast<const float4 *>(R),
        reinterpret_cast<const float4 *>(Q), (float)c, (float)qs);
    return hipGetLastError();
}

__global__ void k_cg_final(int ldb, CgState st) {
    int c = blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= ldb) return;
    double r0 = st.rho0[c];
    st.relres[c] = r0 > 0.0 ? sqrt(st.rho[c] / r0) : 0.0;
}

hipError_t launch_cg_final(int ldb, CgState st, hipStream_t s) {
    k_cg_final<<<(ldb + 63) / 64, 64, 0, s>>>(ldb, st);
    return hipGetLastError();
}

// Section 4.2, eq. (h-spectral): c = U1^T y is a gather of the k_y rows of U1
// that y touches. Writes Cs = g(lambda) .* c (the spectral coefficients,
// g(x) = h(x) - h(0), eq. (aux)) and Cl = lambda .* c, which is L1 U1^T P for
// the first CG product since P0 = y. Storage kinds: fp32 row-major, one or
// two bfloat16 terms in fragment order, FP8 E4M3 codes in fragment order
// with one scale per component (applied here: c is the product with the
// stored U1 itself, and Cs, Cl are written as the coefficients of the codes).
enum { UF_F32 = 0, UF_BF16 = 1, UF_FP8 = 2 };
template <int UF>
__device__ __forceinline__ double u_elem(const void *U, const void *U_lo, size_t o) {
    if (UF == UF_F32) return (double)reinterpret_cast<const float *>(U)[o];
    if (UF == UF_FP8)
        // OCP E4M3 code to fp32 by the gfx950 scaled conversion (scale 1)
        return (double)__builtin_amdgcn_cvt_scalef32_f32_fp8(
            (unsigned)reinterpret_cast<const uint8_t *>(U)[o], 1.0f, 0);
    double v = (double)__uint_as_float((uint32_t)reinterpret_cast<const unsigned short *>(U)[o] << 16);
    if (U_lo) v += (double)__uint_as_float((uint32_t)reinterpret_cast<const unsigned short *>(U_lo)[o] << 16);
    return v;
}

template <int UF>
__global__ __launch_bounds__(kBlock) void k_gather_proj(int B, int ky, const int32_t *ids,
                                                        const float *vals, int64_t N,
                                                        const void *U, const void *U_lo, int rp, int rk,
                                                        int r_use, const double *lam, double alpha,
                                                        int ldb, float *Cs, float *Cl,
                                                        const int32_t *colmap, const double *gv,
                                                        double *Dg, const float *uscale) {
    int k = blockIdx.x * kBlock + threadIdx.x;
    int b = blockIdx.y;  // y row; its solver column is colmap[b] (or b)
    if (k >= rk) return;
    if (colmap && b >= B) return;
    const int col = colmap ? colmap[b] : b;
    double acc = 0.0;
    if (k < r_use && b < B) {
        for (int t = 0; t < ky; ++t) {
            int id = ids[b * ky + t];
            if (id >= 0 && (int64_t)id < N) {
                // fp32 U is row-major; the matrix-core forms are in fragment order
                const size_t o = UF == UF_F32 ? (size_t)id * rp + k : frag_offset(id, k, rp / 32);
                acc += u_elem<UF>(U, U_lo, o) * (double)vals[b * ky + t];
            }
        }
    }
    // the fp8 codes' scale: acc becomes the product with the stored U1, and
    // the coefficients below are those of the codes
    const double sk = UF == UF_FP8 && k < r_use ? (double)uscale[k] : 1.0;
    acc *= sk;
    double lk = k < r_use ? lam[k] : 0.0;
    double h = (1.0 - alpha) / (1.0 - alpha * lk);
    // g of a general filter (Appendix A, eq. (2-aux)) when given, else g_alpha
    double g = gv ? (k < r_use ? gv[k] : 0.0) : h - (1.0 - alpha);
    Cs[(size_t)k * ldb + col] = (float)(g * acc * sk);
    if (Cl) Cl[(size_t)k * ldb + col] = (float)(lk * acc * sk);
    // eigenvector part of y^T Q when the correction follows the sparse product
    if (Dg) Dg[(size_t)k * ldb + col] = alpha / (1.0 - alpha) * lk * acc * acc;
}

hipError_t launch_gather_proj(int B, int ky, const int32_t *ids, const float *vals, int64_t N,
                              const void *U, const void *U_lo, int fmt, int rp, int rk, int r_use,
                              const double *lam, double alpha, int ldb, float *Cs, float *Cl,
                              hipStream_t s, const int32_t *colmap, const double *gv, double *Dg,
                              const float *uscale) {
    if (rk == 0) return hipSuccess;
    if (fmt == UF_FP8 && !uscale) return hipErrorInvalidValue;
    dim3 grid((rk + kBlock - 1) / kBlock, colmap ? B : ldb);
#define HD_GP(UFV)                                                                                               \
    k_gather_proj<UFV><<<grid, kBlock, 0, s>>>(B, ky, ids, vals, N, U, U_lo, rp, rk, r_use, lam, alpha, ldb, Cs, \
                                               Cl, colmap, gv, Dg, uscale)
    if (fmt == UF_FP8) HD_GP(UF_FP8); else if (fmt == UF_BF16) HD_GP(UF_BF16); else HD_GP(UF_F32);
#undef HD_GP
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Continuous batching: a server keeps one solve running over ldb columns and
// lets requests join (admission) and leave (retirement) between iterations.
// Each column is its own CG recurrence, so a request's arithmetic is the same
// whatever else shares the batch.

// A wave per row, lane -> slot t (t fastest, 64 slots per instruction):
// admission takes the lowest free columns, so the slots are mostly runs of
// adjacent columns and a wave's writes to a row coalesce. The slot list is
// staged in LDS once per block (ncols <= 1024) and every index is 32-bit
// within a row (a 64-bit divide per element had made this ALU-bound).
__global__ __launch_bounds__(kBlock) void k_zero_cols(int64_t N, int ldb, float *X, float *R,
                                                      float *P, const int32_t *cols, int ncols) {
    __shared__ int32_t sc[1024];
    for (int t = threadIdx.x; t < ncols; t += kBlock) sc[t] = cols[t];
    __syncthreads();
    const int lane = threadIdx.x % kWave, wr = threadIdx.x / kWave;
    for (int64_t i = (int64_t)blockIdx.x * (kBlock / kWave) + wr; i < N;
         i += (int64_t)gridDim.x * (kBlock / kWave)) {
        const size_t row = vec_index(N, ldb, i, 0);
        for (int t = lane; t < ncols; t += kWave) {
            const size_t o = row + (size_t)sc[t];
            X[o] = 0.f;
            R[o] = 0.f;
            P[o] = 0.f;
        }
    }
}


hipError_t launch_zero_cols(int64_t N, int ldb, float *X, float *R, float *P, const int32_t *cols,
                            int ncols, hipStream_t s) {
    if (ncols == 0 || N == 0) return hipSuccess;
    if (ncols > 1024 || ncols > ldb) return hipErrorInvalidValue;
    const int64_t want = (N + kBlock / kWave - 1) / (kBlock / kWave);
    k_zero_cols<<<(unsigned)(want < 16384 ? want : 16384), kBlock, 0, s>>>(N, ldb, X, R, P, cols, ncols);
    return hipGetLastError();
}

__global__ __launch_bounds__(kScalarThreads) void k_init_cols(int ldb, const double *part, int nblk,
                                                              CgState st, const int32_t *cols,
                                                              const int32_t *maxit, int ncols) {
    const int lane = threadIdx.x % kWave;
    const int c = blockIdx.x * kWave + lane;
    const double rho0 = tile_reduce(part, nblk, ldb, c);
    if (threadIdx.x < kWave) {
        int t = -1;
        for (int q = 0; q < ncols; ++q)
            if (cols[q] == c) t = q;
        if (t >= 0) {
            int act = 0, stat;
            if (rho0 == 0.0) {
                stat = COL_ZERO_RHS;
            } else if (!(rho0 > 0.0) || !isfinite(rho0)) {
                stat = COL_BREAKDOWN;
            } else {
                stat = COL_MAXITER;
                act = maxit[t] > 0 ? 1 : 0;
            }
            st.rho0[c] = rho0 == 0.0 ? 0.0 : rho0;
            st.rho[c] = rho0;
            st.a[c] = 0.0;
            st.beta[c] = 0.0;
            st.relres[c] = rho0 > 0.0 ? 1.0 : 0.0;
            st.active[c] = act;
            st.iters[c] = 0;
            st.status[c] = stat;
            st.maxit[c] = maxit[t];
        }
    }
}

hipError_t launch_init_cols(int ldb, const double *part, int nblk, CgState st, const int32_t *cols,
                            const int32_t *maxit, int ncols, hipStream_t s) {
    if (ncols == 0) return hipSuccess;
    k_init_cols<<<ldb / kWave, kScalarThreads, 0, s>>>(ldb, part, nblk, st, cols, maxit, ncols);
    return hipGetLastError();
}

// Stop columns cols[0..ncols) at once (cancelled requests, or an admission
// that failed): they take no further part in any iteration. Their vectors
// are left as they are; the next admission into a column zeroes it.
__global__ void k_cancel_cols(CgState st, const int32_t *cols, int ncols) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= ncols) return;
    const int c = cols[t];
    st.active[c] = 0;
    st.a[c] = 0.0;
}

hipError_t launch_cancel_cols(CgState st, const int32_t *cols, int ncols, hipStream_t s) {
    if (ncols == 0) return hipSuccess;
    k_cancel_cols<<<(ncols + 63) / 64, 64, 0, s>>>(st, cols, ncols);
    return hipGetLastError();
}

// Xc (N x ldc) and Csc (rk x ldc): slot t of each row takes column cols[t]
// (zero for t >= ncols). A wave per row (the N rows of X, then the rk rows
// of Cs), lane -> slot (64 per instruction): it reads runs of one row of X
// and writes whole rows of Xc; the slot list is staged in LDS.
// iters (nullptr = none): a column with no iteration done takes x = 0 (its
// X may still hold a previous occupant's values, overwritten at its first
// update).
__global__ __launch_bounds__(kBlock) void k_gather_cols(int64_t N, int ldb, const float *X,
                                                        const float *Cs, int rk,
                                                        const int32_t *cols, int ncols, int ldc,
                                                        float *Xc, float *Csc, const int32_t *iters) {
    __shared__ int32_t sc[1024];
    __shared__ bool xz[1024];
    for (int t = threadIdx.x; t < ncols; t += kBlock) {
        sc[t] = cols[t];
        xz[t] = iters && iters[cols[t]] == 0;
    }
    __syncthreads();
    const int lane = threadIdx.x % kWave, wr = threadIdx.x / kWave;
    const int64_t rows = N + (rk > 0 ? rk : 0);
    for (int64_t i = (int64_t)blockIdx.x * (kBlock / kWave) + wr; i < rows;
         i += (int64_t)gridDim.x * (kBlock / kWave)) {
        const bool x = i < N;
        const int64_t r = x ? i : i - N;
        const float *src = (x ? X : Cs) + (size_t)r * (size_t)ldb;
        float *dst = (x ? Xc : Csc) + (size_t)r * (size_t)ldc;
        for (int t = lane; t < ldc; t += kWave) dst[t] = t < ncols && !(x && xz[t]) ? src[sc[t]] : 0.f;
    }
}

hipError_t launch_gather_cols(int64_t N, int ldb, const float *X, const float *Cs, int rk,
                              const int32_t *cols, int ncols, int ldc, float *Xc, float *Csc,
                              hipStream_t s, const int32_t *iters) {
    const int64_t rows = N + (rk > 0 ? rk : 0);
    if (rows == 0 || ldc == 0) return hipSuccess;
    if (ncols > ldc || ldc > 1024) return hipErrorInvalidValue;
    const int64_t want = (rows + kBlock / kWave - 1) / (kBlock / kWave);
    k_gather_cols<<<(unsigned)(want < 16384 ? want : 16384), kBlock, 0, s>>>(N, ldb, X, Cs, rk, cols, ncols, ldc,
                                                                            Xc, Csc, iters);
    return hipGetLastError();
}

}  // namespace hd
