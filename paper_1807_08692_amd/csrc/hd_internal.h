// Internal declarations shared by the C ABI sources (hd_api.cpp: context,
// loaders, batch queries; hd_serve.cpp: the continuous-batching server):
// error reporting, device buffers, per-kernel event timing, the context.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/hd.h"
#include "hd_kernels.h"

namespace hdi {

// Message of the last failure on this thread (returned by hd_last_error).
extern thread_local std::string g_err;

inline int fail(int code, const char *fmt, ...) __attribute__((format(printf, 2, 3)));
inline int fail(int code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define HIP_TRY(call)                                                                   \
    do {                                                                                \
        hipError_t e_ = (call);                                                         \
        if (e_ != hipSuccess)                                                           \
            return fail(e_ == hipErrorOutOfMemory ? HD_ENOMEM : HD_EDEVICE, "%s: %s",   \
                        #call, hipGetErrorString(e_));                                  \
    } while (0)

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    void release() {
        if (p) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
    }
    // Grow-only: keeps the allocation when it is already large enough.
    hipError_t ensure(size_t want) {
        if (want <= bytes && p) return hipSuccess;
        release();
        if (want == 0) want = 256;
        hipError_t e = hipMalloc(&p, want);
        if (e == hipSuccess) bytes = want;
        return e;
    }
    template <class T>
    T *as() const { return reinterpret_cast<T *>(p); }
};

// fp32 -> bfloat16 bit pattern, round to nearest even (inputs are finite).
inline uint16_t bf16_rne_host(float f) {
    uint32_t u;
    std::memcpy(&u, &f, 4);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// OCP FP8 E4M3 (hd_fp8.cpp): round to nearest even with saturation at 448,
// the value of a code, the NaN codes (0x7F, 0xFF), and the quantizer of a
// rows x cols row-major matrix with one scale per column or per row (scale =
// max |a| / 448, 1 for an all-zero line; code = RNE(a / scale)).
uint8_t fp8_e4m3_rne(float x);
float fp8_e4m3_value(uint8_t b);
bool fp8_e4m3_is_nan(uint8_t b);
void fp8_quantize(int64_t rows, int32_t cols, const float *A, bool per_column, uint8_t *codes, float *scales);

// Device address of the fixed scratch array of hd_rank_noalloc on `device`,
// taken once per device (hd_noalloc.hip); called by hd_create.
int noalloc_init(int device);

inline int pow2_at_least(int v) {
    int p = 64;
    while (p < v) p <<= 1;
    return p;
}

// Kernel kinds for the optional per-launch event timing.
enum Kind {
    K_SIM, K_TOPK_Y, K_FILL, K_SCATTER, K_COLSQ, K_SCALAR, K_GATHER, K_UT_P, K_REDUCE_C,
    K_U_C, K_SPMM, K_UPDATE_R, K_UPDATE_XP, K_COMBINE, K_TOPK_RANK,
    K_SPMM_Y,  // the first sparse product, gathering only the rows of y
    K_PERSIST, // the persistent CG kernel (every iteration of a narrow batch)
    K_NKINDS
};
inline const char *const kKindNames[K_NKINDS] = {
    "sim", "topk_y", "fill_zero", "scatter_y", "colsq", "cg_scalar", "gather_proj", "ut_p",
    "reduce_c", "u_c", "spmm", "update_r", "update_xp", "combine", "topk_rank", "spmm_y", "cg_persist"};

struct Timing {
    bool on = false;
    uint32_t mask = ~0u;  // kinds that get events while on
    std::vector<hipEvent_t> pool;
    size_t used = 0;
    struct Pending {
        int kind;
        size_t ev;
        int iter;  // CG iteration the launch belongs to (0 = none)
    };
    std::vector<Pending> pending;
    int tag = 0;  // iteration of the launches being queued
    double total_ms[K_NKINDS] = {};
    int64_t count[K_NKINDS] = {};

    void reset() {
        for (int k = 0; k < K_NKINDS; ++k) {
            total_ms[k] = 0.0;
            count[k] = 0;
        }
        pending.clear();
        used = 0;
    }
    hipError_t begin(hipStream_t s, size_t *idx) {
        if (used + 2 > pool.size()) {
            for (int t = 0; t < 64; ++t) {
                hipEvent_t e;
                hipError_t err = hipEventCreate(&e);
                if (err != hipSuccess) return err;
                pool.push_back(e);
            }
        }
        *idx = used;
        used += 2;
        return hipEventRecord(pool[*idx], s);
    }
    hipError_t end(int kind, size_t idx, hipStream_t s) {
        pending.push_back({kind, idx, tag});
        return hipEventRecord(pool[idx + 1], s);
    }
    // Call after the stream has been synchronised. Launches of iterations
    // after last_iter were queued ahead and returned at once; they are not
    // counted.
    hipError_t harvest(int last_iter) {
        for (auto &pk : pending) {
            if (pk.iter > last_iter) continue;
            float ms = 0.f;
            hipError_t e = hipEventElapsedTime(&ms, pool[pk.ev], pool[pk.ev + 1]);
            if (e != hipSuccess) return e;
            total_ms[pk.kind] += ms;
            count[pk.kind] += 1;
        }
        pending.clear();
        used = 0;
        return hipSuccess;
    }
    void destroy() {
        for (hipEvent_t e : pool) (void)hipEventDestroy(e);
        pool.clear();
    }
};

}  // namespace hdi

using namespace hdi;

struct hd_ctx {
    int device = 0;
    // graph
    int64_t n = 0, nnz = 0;
    DevBuf rowptr, col, val;
    DevBuf cut;  // source-band cut offsets of the sparse product (8 per row)
    // eigenpairs: U (fp32, N x rp) or Ub (bf16, N x rp, rows padded to 16) +
    // UbT (bf16, rp x ldut), both in fragment order (hd::frag_offset); the
    // two-term form stores the lo terms after the hi terms of each; the fp8
    // form keeps E4M3 codes (one byte per element) in the same two layouts
    // and one fp32 scale per component in uscale (rp values)
    int r = 0, rp = 0, u_dtype = HD_F32;
    int64_t ldut = 0;
    DevBuf U, Ub, UbT, lam, uscale;
    // sparsified U1 (SHybrid): by item (CSR) and by component (CSC, rp + 1 pointers)
    DevBuf Usr, Usc, Usv, Ustp, Ustr, Ustv;
    int64_t us_nnz = 0;
    std::vector<double> lam_host;  // the loaded eigenvalues, padded with zeros to rp
    DevBuf gfil;                   // g(lambda) of a general filter
    int eig_outer = 0;             // Rayleigh-Ritz steps of the last hd_compute_eigs
    // descriptors: V (fp32, N x ldv) or Vb (bf16, N x ldv in fragment order,
    // rows padded to 16)
    int d = 0, ldv = 0, v_dtype = HD_F32;
    DevBuf V, Vb, vscale;  // vscale: one fp32 scale per row of fp8 descriptors
    // the one-pass top-K's row sample (items t * stride, hd::topk_sample) of
    // the matrix-core storage forms, in the same layouts: Vsm the sampled
    // descriptors (then, for fp8, their row scales), Usm the sampled
    // item-major U1 rows (hi, then lo for the two-term form); empty when
    // n < hd::kTopkFuseMin or the form is fp32. tsx: per-batch sample scores
    // and sampled rows of x^t
    DevBuf Vsm, Usm, tsx;
    size_t vsm_scale_off = 0, usm_lo_off = 0;  // bytes: fp8 row scales in Vsm, lo terms in Usm
    // solver workspace
    DevBuf X, R, P, Q, Z, Cpart, Cl, Cs, ClT, CsT, PT, part, scal, xbuf, sim, ybuf, topk, err, qsplit;
    int32_t *h_pinned = nullptr;  // [0..128): nact counts by parity, [200]: error flag
    hipEvent_t iter_ev[2] = {nullptr, nullptr};
    DevBuf Dg;  // alpha / (1 - alpha) lambda (U1^T P)^2 per component and column
    DevBuf pre;  // pre-reduced partial sums of the scalar kernels (2 x 64 rows of ldb)
    DevBuf ymask;  // one bit per item: the rows where y (the first P) is nonzero
    hd::CgState st{};
    Timing timing;
    int tune[HD_TUNE_NKEYS] = {0, 0, 0, 0, 0};  // launch parameters (0 = default)
    // persistent CG for narrow batches: 0 off, 1 up to 16 queries, 2 up to 64;
    // the bound on each grid-barrier wait (spins); its barrier words
    int persist_mode = 0;
    long long persist_spin = 1LL << 24;
    DevBuf pbar;

    // the matrix-core storage forms of U1 (fragment order): bf16, two-term bf16, fp8
    bool u_mfma() const { return u_dtype == HD_BF16 || u_dtype == HD_BF16X2 || u_dtype == HD_FP8_E4M3; }
    bool u_fp8() const { return u_dtype == HD_FP8_E4M3; }
    // per-component scales of the fp8 form (null otherwise)
    const float *u_scale() const { return u_fp8() ? uscale.as<float>() : nullptr; }
    bool u_sparse() const { return u_dtype == HD_SPARSE_F32; }
    // second bfloat16 terms of the two-term U1 form (null otherwise)
    const uint16_t *ub_lo() const {
        return u_dtype == HD_BF16X2 ? Ub.as<uint16_t>() + (size_t)((n + 15) / 16 * 16) * rp : nullptr;
    }
    const uint16_t *ubt_lo() const {
        return u_dtype == HD_BF16X2 ? UbT.as<uint16_t>() + (size_t)rp * ldut : nullptr;
    }
    // the stored U1 as the matrix-core kernels' operand: item-major / component-major
    hd::UOperand u_item() const { return hd::UOperand{Ub.p, ub_lo(), u_fp8()}; }
    hd::UOperand u_comp() const { return hd::UOperand{UbT.p, ubt_lo(), u_fp8()}; }
    // storage kind for launch_gather_proj: 0 fp32, 1 bf16 terms, 2 fp8 codes
    int u_fmt() const { return u_fp8() ? 2 : (u_mfma() ? 1 : 0); }
    // descriptors: the stored matrix of the similarity kernels (fp32 V, or the
    // fragment-order bf16 / fp8 Vb) and the fp8 row scales (null otherwise)
    const float *v_scale() const { return v_dtype == HD_FP8_E4M3 ? vscale.as<float>() : nullptr; }
    // launch parameter `key` for solver width ldb (0 = default when unset or
    // not fitting the width)
    int tv(int key, int ldb) const {
        if (key == HD_TUNE_SPMM_BANDS) return hd::band_param_ok(tune[key]) ? tune[key] : 1;
        if (key == HD_TUNE_TOPK_ONEPASS) return tune[key];
        return hd::tile_param_ok(tune[key], ldb) ? tune[key] : 0;
    }
    // the sparse product's source-band count and cut offsets
    int bands() const { return hd::band_param_ok(tune[HD_TUNE_SPMM_BANDS]) ? tune[HD_TUNE_SPMM_BANDS] : 1; }
    const int32_t *cuts() const { return cut.as<int32_t>(); }
    // the one-pass top-K applies to the y step / the ranking (setting 1
    // keeps the two-pass form everywhere)
    const float *vsm_scale() const {
        return v_dtype == HD_FP8_E4M3 ? reinterpret_cast<const float *>(Vsm.as<char>() + vsm_scale_off) : nullptr;
    }
    hd::UOperand u_item_sample() const {
        return hd::UOperand{Usm.p, u_dtype == HD_BF16X2 ? Usm.as<char>() + usm_lo_off : nullptr, u_fp8()};
    }
    bool onepass_y() const { return tune[HD_TUNE_TOPK_ONEPASS] != 1 && Vsm.p != nullptr; }
    bool onepass_rank(int rk) const {
        return tune[HD_TUNE_TOPK_ONEPASS] != 1 && n >= hd::kTopkFuseMin && (rk == 0 || (u_mfma() && Usm.p));
    }
};

namespace hdi {
// A polynomial filter h(x) = sum_{i <= degree} coeffs[i] x^i (Appendix A).
struct Filter {
    int degree;
    const double *coeffs;
};
// Validate and queue the whole query path of hd_query_batch on stream s.
// graph = false: the host watches the stopping test (one iteration of
// lookahead) and returns after queueing the final steps. graph = true: all
// max_iter iterations are queued with no host synchronisation and no event
// or host copy, so the sequence can be captured into a HIP graph; the y-id
// error flag is left in c->err and the per-column results in c->st.
int queue_query(hd_ctx *c, int32_t B, const float *q_desc, const int32_t *y_ids, const float *y_val,
                const hd_query_opts *o, int32_t *rank_ids, float *rank_scores, float *x_out,
                int32_t *y_ids_out, float *y_val_out, hipStream_t s, bool graph, int *last_iter,
                const Filter *flt = nullptr);
}  // namespace hdi

// Launch `call` (a launcher returning hipError_t) as kernel kind `kind`,
// bracketed by timing events when timing is on.
#define LAUNCH(kind, call)                                                        \
    do {                                                                          \
        size_t ev_ = 0;                                                           \
        const bool tm_ = c->timing.on && ((c->timing.mask >> (kind)) & 1u);       \
        if (tm_) HIP_TRY(c->timing.begin(s, &ev_));                               \
        HIP_TRY(call);                                                            \
        if (tm_) HIP_TRY(c->timing.end(kind, ev_, s));                            \
    } while (0)

