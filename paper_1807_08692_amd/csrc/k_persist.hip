// Persistent conjugate gradient for narrow batches (the batching form): one
// kernel runs every CG iteration of a batch of W <= 64 query columns, so a
// batch costs one launch for the whole temporal term instead of about seven
// launches and one host round trip per iteration (Section 5: CG from x0 = 0;
// Section 4.2, eq. (box): the deflated operator, here with fp32 U1 and
// vector-ALU products, which at these widths are bound by the bytes of U1,
// not by arithmetic; eq. (temporal) when r = 0).
//
// Vectors are node-major N x W (W a power of two, 1..64). The blocks are
// co-resident (grid sized from the occupancy) and own contiguous row ranges;
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

struct PersistArgs {
    int64_t N;
    const int64_t *rowptr;
    const int32_t *col;
    const float *val;
    const float *U;  // fp32 item-major N x rp (hybrid), else null
    int rp, rk, r_use;
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

// Column sums of per-lane doubles over the block (lane (slot, c), c = lane % W)
// in a fixed order, written by threads t < W to out[t].
template <int W>
__device__ __forceinline__ void block_colsum(double v, double *out) {
    __shared__ double red[kBlock];
    red[threadIdx.x] = v;
    __syncthreads();
    if (threadIdx.x < W) {
        double s = 0.0;
        for (int j = threadIdx.x; j < kBlock; j += W) s += red[j];
        out[threadIdx.x] = s;
    }
    __syncthreads();
}

template <int W, bool HYB>
__global__ __launch_bounds__(kBlock) void k_cg_persist(PersistArgs A) {
    constexpr int S = kWave / W;      // rows per wave step (lane = slot * W + c)
    constexpr int TR = kBlock / W;    // rows per tile of the vector phases
    extern __shared__ float cl_lds[];  // hybrid: Cl transposed (W x rk: lanes read consecutive k)
    __shared__ float pt[TR][W];        // hybrid: the tile's new p
    const int t = threadIdx.x, lane = t % kWave, wv = t / kWave;
    const int c = lane % W, slot = lane / W;
    const int tc = t % W, tr = t / W;  // tile mapping: row tr, column tc
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
    // phase functions of the last arriving block
    auto last_a = [&](int it) {
        if (t < W) {
            if (it == 1) init_state();
            double gamma = 0.0;
            for (int b = 0; b < G; ++b) gamma += A.gpart[(size_t)b * W + t];
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
        if (t == 0) nact = 0;
        __syncthreads();
        if (t < W) {
            double rn = 0.0;
            for (int b = 0; b < G; ++b) rn += A.rpart[(size_t)b * W + t];
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
            const double ac = st.a[tc], bc = st.beta[tc];
            const int actc = st.active[tc];
            float acc[HYB ? 4 : 1][HYB ? W : 1];
            if (HYB) {
#pragma unroll
                for (int j = 0; j < 4; ++j)
#pragma unroll
                    for (int q = 0; q < W; ++q) acc[j][q] = 0.f;
            }
            for (int64_t t0 = rs; t0 < re; t0 += TR) {
                const int64_t i = t0 + tr;
                float pn = 0.f;
                if (i < re) {
                    const size_t o = (size_t)i * W + tc;
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
                    pt[tr][tc] = pn;
                    __syncthreads();
                    if (t < A.rk / 4) {
                        for (int r = 0; r < TR && t0 + r < re; ++r) {
                            const float4 u = *reinterpret_cast<const float4 *>(A.U + (size_t)(t0 + r) * A.rp + 4 * t);
#pragma unroll
                            for (int q = 0; q < W; ++q) {
                                const float pv = pt[r][q];
                                acc[0][q] += u.x * pv;
                                acc[1][q] += u.y * pv;
                                acc[2][q] += u.z * pv;
                                acc[3][q] += u.w * pv;
                            }
                        }
                    }
                    __syncthreads();
                }
            }
            if (HYB) {
                if (t < A.rk / 4) {
                    float *out = A.Cpart + (size_t)blockIdx.x * A.rk * W + (size_t)(4 * t) * W;
#pragma unroll
                    for (int j = 0; j < 4; ++j)
#pragma unroll
                        for (int q = 0; q < W; ++q) out[j * W + q] = acc[j][q];
                }
                if (!grid_sync(A.ps, gen, noop)) return;
                // ---- C: Cl = L1 sum over blocks (fixed order), spread over the grid ----
                const int ne = A.rk * W;
                for (int e = blockIdx.x * kBlock + t; e < ne; e += G * kBlock) {
                    const int k = e / W;
                    double s = 0.0;
                    for (int b = 0; b < G; ++b) s += (double)A.Cpart[(size_t)b * ne + e];
                    A.Cl[e] = k < A.r_use ? (float)(A.lam[k] * s) : 0.f;
                }
            }
            if (!grid_sync(A.ps, gen, noop)) return;
        }

        // ---- A: q = (z - alpha S p) / (1 - alpha), z = p (+ alpha U1 Cl); gamma partials ----
        if (HYB) {
            for (int e = t; e < A.rk * W; e += kBlock) cl_lds[(e % W) * A.rk + e / W] = A.Cl[e];
            __syncthreads();
        }
        double g = 0.0;
        for (int64_t i0 = rs + (int64_t)wv * S; i0 < re; i0 += 4 * S) {
            const int64_t i = i0 + slot;
            float zc = 0.f;
            if (HYB) {
                // the U1 Cl entries of the step's rows: lanes over components
                for (int s2 = 0; s2 < S && i0 + s2 < re; ++s2) {
                    const float *urow = A.U + (size_t)(i0 + s2) * A.rp;
                    float part[W];
#pragma unroll
                    for (int q = 0; q < W; ++q) part[q] = 0.f;
                    for (int k = lane; k < A.rk; k += kWave) {
                        const float u = urow[k];
#pragma unroll
                        for (int q = 0; q < W; ++q) part[q] += u * cl_lds[q * A.rk + k];
                    }
#pragma unroll
                    for (int q = 0; q < W; ++q) {
                        const float v = wave_sum_f32(part[q]);
                        if (slot == s2 && c == q) zc = v;
                    }
                }
            }
            if (i < re) {
                const size_t o = (size_t)i * W + c;
                const float p = A.P[o];
                float acc = 0.f;
                for (int64_t e = A.rowptr[i]; e < A.rowptr[i + 1]; ++e)
                    acc += A.val[e] * A.P[(size_t)A.col[e] * W + c];
                const float z = HYB ? p + A.alpha * zc : p;
                const float q = (z - A.alpha * acc) / A.oma;
                A.Q[o] = q;
                g += (double)p * (double)q;
            }
        }
        block_colsum<W>(g, A.gpart + (size_t)blockIdx.x * W);
        if (!grid_sync(A.ps, gen, [&] { last_a(it); })) return;

        // ---- R: r -= a q; rho' partials; stopping test ----
        {
            const double ac = st.a[c];
            double rr = 0.0;
            for (int64_t i0 = rs + (int64_t)wv * S; i0 < re; i0 += 4 * S) {
                const int64_t i = i0 + slot;
                if (i < re) {
                    const size_t o = (size_t)i * W + c;
                    float r = A.R[o];
                    if (ac != 0.0) r = (float)((double)r - ac * (double)A.Q[o]);
                    A.R[o] = r;
                    rr += (double)r * (double)r;
                }
            }
            block_colsum<W>(rr, A.rpart + (size_t)blockIdx.x * W);
        }
        if (!grid_sync(A.ps, gen, last_b)) return;
        if (__hip_atomic_load(&A.ps.w[3], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0u) break;
    }
    // ---- the last step of x: x += a p ----
    const double ac = st.a[tc];
    if (ac != 0.0) {
        for (int64_t t0 = rs; t0 < re; t0 += TR) {
            const int64_t i = t0 + tr;
            if (i < re) {
                const size_t o = (size_t)i * W + tc;
                A.X[o] = (float)((double)A.X[o] + ac * (double)A.P[o]);
            }
        }
    }
}

// x[b][i] = (U1 Cs)[i][b] + X[i][b] for b < B (query-major, row stride ldx),
// narrow X (N x W): one wave per item row, lanes over components, Cs staged
// in LDS (rk x W); plain CG (rk = 0) is the transpose of X.
template <int W>
__global__ __launch_bounds__(kBlock) void k_combine_narrow(int64_t N, int B, const float *__restrict__ U, int rp,
                                                           int rk, const float *__restrict__ Cs,
                                                           const float *__restrict__ X, float *__restrict__ x,
                                                           int64_t ldx) {
    extern __shared__ float cs_lds[];  // Cs transposed (W x rk)
    const int t = threadIdx.x, lane = t % kWave;
    for (int e = t; e < rk * W; e += kBlock) cs_lds[(e % W) * rk + e / W] = Cs[e];
    __syncthreads();
    const int64_t nw = (int64_t)gridDim.x * (kBlock / kWave);
    for (int64_t i = (int64_t)blockIdx.x * (kBlock / kWave) + t / kWave; i < N; i += nw) {
        float part[W];
#pragma unroll
        for (int q = 0; q < W; ++q) part[q] = 0.f;
        for (int k = lane; k < rk; k += kWave) {
            const float u = U[(size_t)i * rp + k];
#pragma unroll
            for (int q = 0; q < W; ++q) part[q] += u * cs_lds[q * rk + k];
        }
#pragma unroll
        for (int q = 0; q < W; ++q) {
            const float v = rk > 0 ? wave_sum_f32(part[q]) : 0.f;
            if (lane == q && q < B) x[(size_t)q * ldx + i] = v + X[(size_t)i * W + q];
        }
    }
}

bool persist_width_ok(int W, int rk) {
    if (W < 1 || W > 64 || (W & (W - 1)) != 0) return false;
    if (rk == 0) return true;
    return W <= 16 && rk % 32 == 0 && rk <= 1024;
}

size_t persist_lds_bytes(int W, int rk) { return (size_t)rk * W * sizeof(float); }

template <int W, bool HYB>
static hipError_t grid_of(size_t lds, int *grid) {
    int dev = 0, per_cu = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, dev);
    if (e != hipSuccess) return e;
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, k_cg_persist<W, HYB>, kBlock, lds);
    if (e != hipSuccess) return e;
    if (per_cu < 1) return hipErrorInvalidConfiguration;
    // at most two blocks per compute unit: the phases are short, and a
    // barrier's cost grows with the number of blocks
    *grid = prop.multiProcessorCount * (per_cu < 2 ? per_cu : 2);
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
    // no more blocks than rows of work: a block covers at least one wave step
    const int64_t step = 4 * (kWave / W);
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
            case 1: k_cg_persist<1, true><<<grid, kBlock, lds, s>>>(a); break;
            case 2: k_cg_persist<2, true><<<grid, kBlock, lds, s>>>(a); break;
            case 4: k_cg_persist<4, true><<<grid, kBlock, lds, s>>>(a); break;
            case 8: k_cg_persist<8, true><<<grid, kBlock, lds, s>>>(a); break;
            default: k_cg_persist<16, true><<<grid, kBlock, lds, s>>>(a); break;
        }
    } else {
        switch (W) {
            case 1: k_cg_persist<1, false><<<grid, kBlock, 0, s>>>(a); break;
            case 2: k_cg_persist<2, false><<<grid, kBlock, 0, s>>>(a); break;
            case 4: k_cg_persist<4, false><<<grid, kBlock, 0, s>>>(a); break;
            case 8: k_cg_persist<8, false><<<grid, kBlock, 0, s>>>(a); break;
            case 16: k_cg_persist<16, false><<<grid, kBlock, 0, s>>>(a); break;
            case 32: k_cg_persist<32, false><<<grid, kBlock, 0, s>>>(a); break;
            default: k_cg_persist<64, false><<<grid, kBlock, 0, s>>>(a); break;
        }
    }
    return hipGetLastError();
}

hipError_t launch_combine_narrow(int W, int64_t N, int B, const float *U, int rp, int rk, const float *Cs,
                                 const float *X, float *x, int64_t ldx, hipStream_t s) {
    if (W < 1 || W > 64 || B < 1 || B > W) return hipErrorInvalidValue;
    if (rk > 0 && !persist_width_ok(W, rk)) return hipErrorInvalidValue;
    const int64_t want = (N + 3) / 4;
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
