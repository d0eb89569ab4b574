// Persistent conjugate gradient for narrow batches (the batching form): one
// kernel runs every CG iteration of a batch of W <= 64 query columns, so a
// batch costs one launch for the whole temporal term instead of about seven
// launches and one host round trip per iteration (Section 5: CG from x0 = 0;
// Section 4.2, eq. (box): the deflated operator, here with fp32 U1 and
// vector-ALU products, which at these widths are bound by the bytes of U1,
// not by arithmetic; eq. (temporal) when r = 0).
//
// Vectors are node-major N x W (W a power of two, 1..64). Blocks of 1024
// threads (16 waves), at most two per compute unit, are co-resident (grid
// sized from the occupancy, and to about four sparse-product rows per wave
// on small graphs) and own contiguous row ranges;
// phases are separated by grid barriers. A barrier's last arriving block
// performs the phase's scalar work (the fixed-order reductions of the
// per-block partial sums, the step sizes and the stopping test) before it
// releases the others, so every scalar is computed once, in an order that
// depends only on the grid size. Each barrier wait is bounded: past the
// limit the block sets an abort flag and every block returns, so the kernel
// always ends; the host then reports the failure.
//
// One iteration, per column c (the same recurrence as k_cg.hip):
//   P:  x += a p ; p = r + beta p (active columns)      [U1^T p partials]
//   C:  Cl = L1 (U1^T p)                                  (hybrid)
//   A:  z = p + alpha U1 Cl ; q = (z - alpha S p) / (1 - alpha) ; gamma = p^T q
//       -> a = rho / gamma, or breakdown
//   R:  r -= a q ; rho' = r^T r -> stopping test, beta = rho' / rho
// Iteration 1 starts from p = y with Cl = L1 U1^T y from the spectral gather,
// and after the last iteration only x += a p remains.
//
// At a million items the sparse product's neighbour gathers are random, and
// their count (one per nonzero), not their width, sets its time: a narrow
// batch costs about as much per product as 64 columns. Each wave therefore
// keeps several gathers in flight (one row per wave, the row's nonzeros
// spread over the lanes), and the kernel saves the launches and host round
// trips of the multi-kernel path rather than bytes.
#include "hd_device.h"
#include "hd_kernels.h"

namespace hd {

enum { PC_CONVERGED = 0, PC_MAXITER = 1, PC_ZERO_RHS = 2, PC_BREAKDOWN = 3 };

// Barrier words: [0] arrivals, [1] generation, [2] abort, [3] all columns stopped.
struct PersistSync {
    unsigned *w;
    long long spin_limit;
    int32_t *err;  // err[1] = 1 when a wait ran past the limit
};

// Grid barrier with a phase function run by the last block to arrive.
// Returns false when the run was aborted (the caller returns at once).
template <class Last>
__device__ __forceinline__ bool grid_sync(const PersistSync &ps, unsigned &gen, Last last) {
    __shared__ int sh_last, sh_abort;
    __syncthreads();  // this block's stores are complete
    if (threadIdx.x == 0) {
        sh_last = 0;
        sh_abort = 0;
        __threadfence();  // release them at device scope
        const unsigned prev = __hip_atomic_fetch_add(&ps.w[0], 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
        if (prev == gridDim.x - 1) {
            __hip_atomic_store(&ps.w[0], 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            sh_last = 1;
        } else {
            long long spins = 0;
            // relaxed polling; the fence after the loop acquires
            while (__hip_atomic_load(&ps.w[1], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == gen) {
                if (__hip_atomic_load(&ps.w[2], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u ||
                    ++spins > ps.spin_limit) {
                    __hip_atomic_store(&ps.w[2], 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    atomicOr(&ps.err[1], 1);
                    sh_abort = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __threadfence();  // acquire what the other blocks released
    }
    __syncthreads();
    if (sh_abort) return false;
    if (sh_last) {
        last();
        __syncthreads();
        if (threadIdx.x == 0) {
            __threadfence();
            __hip_atomic_store(&ps.w[1], gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
    }
    ++gen;
    return true;
}

// Sum of a float over the 64 lanes (fixed butterfly order; every lane gets it).
__device__ __forceinline__ float wave_sum_f32(float v) {
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

constexpr int kPB = 1024;          // threads per block of the persistent kernel
constexpr int kPW = kPB / kWave;   // its waves

struct PersistArgs {
    int64_t N;
    const int64_t *rowptr;
    const int32_t *col;
    const float *val;
    const float *U;  // fp32 item-major N x rp (hybrid), else null
    int rp, rk, r_use;
    int ngr;         // hybrid: row groups of the U1^T p partials (a power of two)
    const double *lam;
    float alpha, oma;
    float *X, *R, *P, *Q;  // N x W
    float *Cl;             // rk x W: L1 U1^T y on entry, then L1 U1^T p
    float *Cpart;          // grid x rk x W
    double *gpart, *rpart; // grid x W
    const double *yn;      // W values: y^T y per column (columns >= B hold 0)
    CgState st;            // W entries
    int B, max_iter;
    double tol;
    int64_t rb;            // rows per block
    PersistSync ps;
};

// Column sums over the block of per-thread doubles, thread t holding column
// t % W: a fixed butterfly over the lanes of each wave with the same column,
// then the waves in order. The result is valid in threads t < W (column t).
template <int W>
__device__ __forceinline__ double block_colsum(double v) {
    __shared__ double red[kPW][W];
    for (int off = W; off < kWave; off <<= 1) v += __shfl_xor(v, off, kWave);
    const int lane = threadIdx.x % kWave, wv = threadIdx.x / kWave;
    if (lane < W) red[wv][lane] = v;
    __syncthreads();
    double s = 0.0;
    if (threadIdx.x < W)
        for (int j = 0; j < kPW; ++j) s += red[j][threadIdx.x];
    __syncthreads();
    return s;
}

// Thread t's share of a column sum over the grid's per-block partials
// part[b][t % W]: blocks t / W, t / W + kPB / W, ... in order (combined by
// block_colsum, so the whole sum has a fixed order for a given grid).
template <int W>
__device__ __forceinline__ double grid_partials(const double *part, int G) {
    const int c = threadIdx.x % W;
    double s = 0.0;
#pragma unroll 4
    for (int b = threadIdx.x / W; b < G; b += kPB / W) s += part[(size_t)b * W + c];
    return s;
}

// Thread layout: column c = t % W in every phase. Vector phases: tiles of
// kPB / W rows, row t / W of the tile. Sparse product: one row per wave,
// lane (j, c) taking the row's nonzeros j, j + 64 / W, ... (kWave / W slots,
// several gathers per slot in flight), summed over the slots by a fixed
// butterfly. Hybrid U1^T p partials: thread (kq, g) takes components
// 2 kq and 2 kq + 1 and the tile rows g, g + ngr, ..., then the ngr group
// partials are summed by a fixed pairwise tree in LDS.
template <int W, bool HYB>
__global__ __launch_bounds__(kPB) void k_cg_persist(PersistArgs A) {
    constexpr int TR = kPB / W;                 // rows per tile of the vector phases
    constexpr int NJ = kWave / W;               // nonzero slots per wave
    constexpr int UNR = NJ >= 16 ? 1 : 16 / NJ;  // gathers per slot in flight (16 per wave)
    extern __shared__ float dyn_lds[];          // hybrid: Cl^T (W x rk) in A; ngr x rk x W in P
    __shared__ float pt[HYB ? TR : 1][W];       // hybrid: the tile's new p
    const int t = threadIdx.x, lane = t % kWave, wv = t / kWave;
    const int c = t % W, tr = t / W, j = lane / W;
    const int64_t rs = (int64_t)blockIdx.x * A.rb;
    const int64_t re = rs + A.rb < A.N ? rs + A.rb : A.N;
    const int G = gridDim.x;
    CgState st = A.st;
    unsigned gen = 0;

    // the column state from y^T y (thread t < W: column t)
    auto init_state = [&]() {
        const double r0 = A.yn[t];
        int act = 0, stat;
        if (t >= A.B || r0 == 0.0) {
            stat = PC_ZERO_RHS;
        } else if (!(r0 > 0.0) || !isfinite(r0)) {
            stat = PC_BREAKDOWN;
        } else {
            stat = PC_MAXITER;
            act = A.max_iter > 0;
        }
        st.rho0[t] = t < A.B ? r0 : 0.0;
        st.rho[t] = st.rho0[t];
        st.a[t] = 0.0;
        st.beta[t] = 0.0;
        st.relres[t] = st.rho0[t] > 0.0 ? 1.0 : 0.0;
        st.active[t] = act;
        st.iters[t] = 0;
        st.status[t] = stat;
    };
    if (A.max_iter <= 0) {  // no product: x = 0, the state only
        if (blockIdx.x == 0 && t < W) init_state();
        return;
    }
    // phase functions of the last arriving block (every thread calls them)
    auto last_a = [&](int it) {
        const double gamma = block_colsum<W>(grid_partials<W>(A.gpart, G));
        if (t < W) {
            if (it == 1) init_state();
            double a = 0.0;
            if (st.active[t]) {
                if (!(gamma > 0.0) || !isfinite(gamma)) {
                    st.status[t] = PC_BREAKDOWN;
                    st.active[t] = 0;
                } else {
                    a = st.rho[t] / gamma;
                }
            }
            st.a[t] = a;
        }
    };
    __shared__ int nact;
    auto last_b = [&]() {
        const double rn = block_colsum<W>(grid_partials<W>(A.rpart, G));
        if (t == 0) nact = 0;
        __syncthreads();
        if (t < W) {
            if (st.active[t]) {
                st.iters[t] += 1;
                if (sqrt(rn / st.rho0[t]) <= A.tol) {
                    st.status[t] = PC_CONVERGED;
                    st.active[t] = 0;
                } else {
                    st.beta[t] = rn / st.rho[t];
                    atomicAdd(&nact, 1);
                }
                st.rho[t] = rn;
            }
        }
        __syncthreads();
        if (t == 0) A.ps.w[3] = nact == 0 ? 1u : 0u;
    };
    auto noop = [] {};

    for (int it = 1; it <= A.max_iter; ++it) {
        if (it > 1) {
            // ---- P: x += a p, p = r + beta p; hybrid: partial U1^T p ----
            const double ac = st.a[c], bc = st.beta[c];
            const int actc = st.active[c];
            const int kq2 = HYB ? A.rk / 2 : 1;
            const int kq = t % kq2, grp = t / kq2;
            const bool gact = HYB && grp < A.ngr;
            float acc[HYB ? 2 : 1][HYB ? W : 1];
            if (HYB) {
#pragma unroll
                for (int u = 0; u < 2; ++u)
#pragma unroll
                    for (int q = 0; q < W; ++q) acc[u][q] = 0.f;
            }
            for (int64_t t0 = rs; t0 < re; t0 += TR) {
                const int64_t i = t0 + tr;
                float pn = 0.f;
                if (i < re) {
                    const size_t o = (size_t)i * W + c;
                    float x = A.X[o], p = A.P[o];
                    if (ac != 0.0) x = (float)((double)x + ac * (double)p);
                    if (actc) {
                        p = (float)((double)A.R[o] + bc * (double)p);
                        A.P[o] = p;
                    }
                    A.X[o] = x;
                    pn = p;
                }
                if (HYB) {
                    pt[tr][c] = pn;
                    __syncthreads();
                    if (gact) {
                        const int nr = re - t0 < TR ? (int)(re - t0) : TR;
                        for (int r = grp; r < nr; r += A.ngr) {
                            const float2 u = *reinterpret_cast<const float2 *>(A.U + (size_t)(t0 + r) * A.rp + 2 * kq);
#pragma unroll
                            for (int q = 0; q < W; ++q) {
                                const float pv = pt[r][q];
                                acc[0][q] += u.x * pv;
                                acc[1][q] += u.y * pv;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            if (HYB) {
                // the ngr group partials: a fixed pairwise tree in LDS
                const int one = A.rk * W;
                if (gact) {
#pragma unroll
                    for (int u = 0; u < 2; ++u)
#pragma unroll
                        for (int q = 0; q < W; ++q) dyn_lds[(size_t)grp * one + (2 * kq + u) * W + q] = acc[u][q];
                }
                __syncthreads();
                for (int h = A.ngr / 2; h >= 1; h /= 2) {
                    const int ne = h * one;
                    for (int e = t; e < ne; e += kPB) dyn_lds[e] += dyn_lds[e + ne];
                    __syncthreads();
                }
                float *out = A.Cpart + (size_t)blockIdx.x * one;
                for (int e = t; e < one; e += kPB) out[e] = dyn_lds[e];
                if (!grid_sync(A.ps, gen, noop)) return;
                // ---- C: Cl = L1 sum over blocks (fixed order), spread over the grid ----
                for (int e = blockIdx.x * kPB + t; e < one; e += G * kPB) {
                    const int k = e / W;
                    double s = 0.0;
#pragma unroll 4
                    for (int b = 0; b < G; ++b) s += (double)A.Cpart[(size_t)b * one + e];
                    A.Cl[e] = k < A.r_use ? (float)(A.lam[k] * s) : 0.f;
                }
            }
            if (!grid_sync(A.ps, gen, noop)) return;
        }

        // ---- A: q = (z - alpha S p) / (1 - alpha), z = p (+ alpha U1 Cl); gamma partials ----
        if (HYB) {
            for (int e = t; e < A.rk * W; e += kPB) dyn_lds[(e % W) * A.rk + e / W] = A.Cl[e];
            __syncthreads();
        }
        double g = 0.0;
        for (int64_t i = rs + wv; i < re; i += kPW) {
            float zc = 0.f;
            if (HYB) {
                // the U1 Cl entries of row i: lanes over components
                const float *urow = A.U + (size_t)i * A.rp;
                float part[W];
#pragma unroll
                for (int q = 0; q < W; ++q) part[q] = 0.f;
                for (int k = lane; k < A.rk; k += kWave) {
                    const float u = urow[k];
#pragma unroll
                    for (int q = 0; q < W; ++q) part[q] += u * dyn_lds[q * A.rk + k];
                }
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const float v = wave_sum_f32(part[q]);
                    if (c == q) zc = v;
                }
            }
            const int64_t beg = A.rowptr[i], end = A.rowptr[i + 1];
            float acc = 0.f;
            // 64 (column id, value) pairs of the row per coalesced load; slot
            // j takes pairs j, j + NJ, ... of each chunk (its nonzeros
            // beg + j, beg + j + NJ, ... in order)
            for (int64_t eb = beg; eb < end; eb += kWave) {
                const int64_t me = eb + lane;
                const int cidx = me < end ? A.col[me] : 0;
                const float cv = me < end ? A.val[me] : 0.f;
                const int cnt = end - eb < kWave ? (int)(end - eb) : kWave;
                if (NJ == kWave) {  // one pair per lane
                    if (lane < cnt) acc += cv * A.P[(size_t)cidx * W + c];
                    continue;
                }
                for (int t0 = 0; t0 < cnt; t0 += NJ * UNR) {
                    float pp[UNR];
#pragma unroll
                    for (int u = 0; u < UNR; ++u) {
                        const int tt = t0 + u * NJ + j;
                        // NJ == 1: the pair index is the same in every lane
                        const int jc = NJ == 1 ? bcast_i(cidx, (t0 + u) & (kWave - 1))
                                               : __shfl(cidx, tt & (kWave - 1), kWave);
                        pp[u] = tt < cnt ? A.P[(size_t)jc * W + c] : 0.f;
                    }
#pragma unroll
                    for (int u = 0; u < UNR; ++u) {
                        const int tt = t0 + u * NJ + j;
                        const float v = NJ == 1 ? bcast_f(cv, (t0 + u) & (kWave - 1))
                                                : __shfl(cv, tt & (kWave - 1), kWave);
                        if (tt < cnt) acc += v * pp[u];
                    }
                }
            }
            for (int off = W; off < kWave; off <<= 1) acc += __shfl_xor(acc, off, kWave);
            if (j == 0) {
                const size_t o = (size_t)i * W + c;
                const float p = A.P[o];
                const float z = HYB ? p + A.alpha * zc : p;
                const float q = (z - A.alpha * acc) / A.oma;
                A.Q[o] = q;
                g += (double)p * (double)q;
            }
        }
        {
            const double gs = block_colsum<W>(g);
            if (t < W) A.gpart[(size_t)blockIdx.x * W + t] = gs;
        }
        if (!grid_sync(A.ps, gen, [&] { last_a(it); })) return;

        // ---- R: r -= a q; rho' partials; stopping test ----
        {
            const double ac = st.a[c];
            double rr = 0.0;
            for (int64_t t0 = rs; t0 < re; t0 += TR) {
                const int64_t i = t0 + tr;
                if (i < re) {
                    const size_t o = (size_t)i * W + c;
                    float r = A.R[o];
                    if (ac != 0.0) r = (float)((double)r - ac * (double)A.Q[o]);
                    A.R[o] = r;
                    rr += (double)r * (double)r;
                }
            }
            const double rsum = block_colsum<W>(rr);
            if (t < W) A.rpart[(size_t)blockIdx.x * W + t] = rsum;
        }
        if (!grid_sync(A.ps, gen, last_b)) return;
        if (__hip_atomic_load(&A.ps.w[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
    }
    // ---- the last step of x: x += a p ----
    const double ac = st.a[c];
    if (ac != 0.0) {
        for (int64_t t0 = rs; t0 < re; t0 += TR) {
            const int64_t i = t0 + tr;
            if (i < re) {
                const size_t o = (size_t)i * W + c;
                A.X[o] = (float)((double)A.X[o] + ac * (double)A.P[o]);
            }
        }
    }
}

// x[b][i] = X[i][b] + (U1 Cs)[i][b] for b < B (query-major, row stride ldx),
// narrow X (N x W), in tiles of 64 rows: the tile of X read whole, each
// row's U1 Cs by one wave (lanes over components, Cs staged in LDS as
// rk x W transposed), then x written row-contiguous per column.
template <int W>
__global__ __launch_bounds__(kBlock) void k_combine_narrow(int64_t N, int B, const float *__restrict__ U, int rp,
                                                           int rk, const float *__restrict__ Cs,
                                                           const float *__restrict__ X, float *__restrict__ x,
                                                           int64_t ldx) {
    extern __shared__ float cs_lds[];  // Cs transposed (W x rk)
    __shared__ float T[W][65];
    const int t = threadIdx.x, lane = t % kWave, wv = t / kWave;
    for (int e = t; e < rk * W; e += kBlock) cs_lds[(e % W) * rk + e / W] = Cs[e];
    for (int64_t i0 = (int64_t)blockIdx.x * 64; i0 < N; i0 += (int64_t)gridDim.x * 64) {
        __syncthreads();  // Cs staged; the previous tile written out
        for (int e = t; e < 64 * W; e += kBlock) {
            const int r = e / W, q = e % W;
            const int64_t i = i0 + r;
            T[q][r] = i < N ? X[(size_t)i * W + q] : 0.f;
        }
        __syncthreads();
        if (rk > 0) {
            for (int r = wv; r < 64 && i0 + r < N; r += kBlock / kWave) {
                const float *urow = U + (size_t)(i0 + r) * rp;
                float part[W];
#pragma unroll
                for (int q = 0; q < W; ++q) part[q] = 0.f;
                for (int k = lane; k < rk; k += kWave) {
                    const float u = urow[k];
#pragma unroll
                    for (int q = 0; q < W; ++q) part[q] += u * cs_lds[q * rk + k];
                }
#pragma unroll
                for (int q = 0; q < W; ++q) {
                    const float v = wave_sum_f32(part[q]);
                    if (lane == q) T[q][r] += v;
                }
            }
            __syncthreads();
        }
        for (int e = t; e < 64 * B; e += kBlock) {
            const int q = e / 64, r = e % 64;
            const int64_t i = i0 + r;
            if (i < N) x[(size_t)q * ldx + i] = T[q][r];
        }
    }
}

bool persist_width_ok(int W, int rk) {
    if (W < 1 || W > 64 || (W & (W - 1)) != 0) return false;
    if (rk == 0) return true;
    return W <= 16 && rk % 32 == 0 && rk <= 1024;
}

// Row groups of the hybrid's U1^T p partials: the largest power of two that
// the block's threads (rk / 2 per group) and an LDS share of
// max(rk W floats, 32 KiB) allow.
static int persist_ngr(int W, int rk) {
    if (rk <= 0) return 1;
    const int by_threads = kPB / (rk / 2);
    const size_t one = (size_t)rk * W * sizeof(float);
    const size_t cap = one > 32768 ? one : 32768;
    const int by_lds = (int)(cap / one);
    const int m = by_threads < by_lds ? by_threads : by_lds;
    int p = 1;
    while (p * 2 <= m) p *= 2;
    return p;
}

size_t persist_lds_bytes(int W, int rk) { return (size_t)persist_ngr(W, rk) * rk * W * sizeof(float); }

template <int W, bool HYB>
static hipError_t grid_of(size_t lds, int *grid) {
    int dev = 0, per_cu = 0, cus = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cg_persist<W, HYB>, kPB, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    // at most two blocks per compute unit: the phases are short, and a
    // barrier's cost grows with the number of blocks
    *grid = cus * (per_cu < 2 ? per_cu : 2);
    return hipSuccess;
}

int persist_grid(int W, int rk, int64_t N) {
    int g = 0;
    const size_t lds = persist_lds_bytes(W, rk);
    hipError_t e = hipErrorInvalidValue;
    if (rk > 0) {
        switch (W) {  // the hybrid takes W <= 16 (persist_width_ok)
            case 1: e = grid_of<1, true>(lds, &g); break;
            case 2: e = grid_of<2, true>(lds, &g); break;
            case 4: e = grid_of<4, true>(lds, &g); break;
            case 8: e = grid_of<8, true>(lds, &g); break;
            case 16: e = grid_of<16, true>(lds, &g); break;
            default: break;
        }
    } else {
        switch (W) {
            case 1: e = grid_of<1, false>(lds, &g); break;
            case 2: e = grid_of<2, false>(lds, &g); break;
            case 4: e = grid_of<4, false>(lds, &g); break;
            case 8: e = grid_of<8, false>(lds, &g); break;
            case 16: e = grid_of<16, false>(lds, &g); break;
            case 32: e = grid_of<32, false>(lds, &g); break;
            case 64: e = grid_of<64, false>(lds, &g); break;
            default: break;
        }
    }
    if (e != hipSuccess || g < 1) return 0;
    // no more blocks than give each wave about four rows of the sparse
    // product (fewer blocks: cheaper barriers on small graphs)
    const int64_t step = 4 * kPW;
    const int64_t need = (N + step - 1) / step;
    return need < g ? (int)(need > 0 ? need : 1) : g;
}

hipError_t launch_cg_persist(int W, int grid, int64_t N, const int64_t *rowptr, const int32_t *col,
                             const float *val, const float *U, int rp, int rk, int r_use, const double *lam,
                             double alpha, float *X, float *R, float *P, float *Q, float *Cl, float *Cpart,
                             double *gpart, double *rpart, const double *yn, CgState st, int B, int max_iter,
                             double tol, unsigned *sync_words, long long spin_limit, int32_t *err,
                             hipStream_t s) {
    if (!persist_width_ok(W, rk) || grid < 1 || B < 1 || B > W) return hipErrorInvalidValue;
    PersistArgs a;
    a.N = N;
    a.rowptr = rowptr;
    a.col = col;
    a.val = val;
    a.U = U;
    a.rp = rp;
    a.rk = rk;
    a.r_use = r_use;
    a.ngr = persist_ngr(W, rk);
    a.lam = lam;
    a.alpha = (float)alpha;
    a.oma = (float)(1.0 - alpha);
    a.X = X;
    a.R = R;
    a.P = P;
    a.Q = Q;
    a.Cl = Cl;
    a.Cpart = Cpart;
    a.gpart = gpart;
    a.rpart = rpart;
    a.yn = yn;
    a.st = st;
    a.B = B;
    a.max_iter = max_iter;
    a.tol = tol;
    a.rb = (N + grid - 1) / grid;
    a.ps = PersistSync{sync_words, spin_limit, err};
    const size_t lds = persist_lds_bytes(W, rk);
    if (rk > 0) {
        switch (W) {  // W <= 16 (checked above)
            case 1: k_cg_persist<1, true><<<grid, kPB, lds, s>>>(a); break;
            case 2: k_cg_persist<2, true><<<grid, kPB, lds, s>>>(a); break;
            case 4: k_cg_persist<4, true><<<grid, kPB, lds, s>>>(a); break;
            case 8: k_cg_persist<8, true><<<grid, kPB, lds, s>>>(a); break;
            default: k_cg_persist<16, true><<<grid, kPB, lds, s>>>(a); break;
        }
    } else {
        switch (W) {
            case 1: k_cg_persist<1, false><<<grid, kPB, 0, s>>>(a); break;
            case 2: k_cg_persist<2, false><<<grid, kPB, 0, s>>>(a); break;
            case 4: k_cg_persist<4, false><<<grid, kPB, 0, s>>>(a); break;
            case 8: k_cg_persist<8, false><<<grid, kPB, 0, s>>>(a); break;
            case 16: k_cg_persist<16, false><<<grid, kPB, 0, s>>>(a); break;
            case 32: k_cg_persist<32, false><<<grid, kPB, 0, s>>>(a); break;
            default: k_cg_persist<64, false><<<grid, kPB, 0, s>>>(a); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_combine_narrow(int W, int64_t N, int B, const float *U, int rp, int rk, const float *Cs,
                                 const float *X, float *x, int64_t ldx, hipStream_t s) {
    if (W < 1 || W > 64 || B < 1 || B > W) return hipErrorInvalidValue;
    if (rk > 0 && !persist_width_ok(W, rk)) return hipErrorInvalidValue;
    const int64_t want = (N + 63) / 64;
    const unsigned grid = (unsigned)(want < 4096 ? (want > 0 ? want : 1) : 4096);
    const size_t lds = (size_t)rk * W * sizeof(float);
#define HD_CN(WV) \
    case WV: k_combine_narrow<WV><<<grid, kBlock, lds, s>>>(N, B, U, rp, rk, Cs, X, x, ldx); break;
    switch (W) {
        HD_CN(1) HD_CN(2) HD_CN(4) HD_CN(8) HD_CN(16) HD_CN(32) HD_CN(64)
        default: return hipErrorInvalidValue;
    }
#undef HD_CN
    return hipGetLastError();
}

}  // namespace hd
