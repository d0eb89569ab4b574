// C ABI of the library (declared in include/hd.h): argument checking, device
// memory of the context, and the host-side schedule of one query batch.
//
// Schedule of hd_query_batch (one HIP stream):
//   1. y         : similarity product + top-k_y + cube    (k_sim, k_topk)
//   2. spectral  : c = U1^T y by gather; Cs = g(L1) c     (k_gather_proj)
//   3. temporal  : per iteration  [U1^T P -> reduce]      (k_ut_p, k_reduce_c)
//                                 [Z = P + a U1 L1 U1^T P] (k_u_c)
//                                 Q = (Z - a S P)/(1 - a)  (k_spmm)
//                                 scalars, R, X, P updates (k_cg_*)
//                  stopping test read back once per iteration
//   4. x = U1 Cs + X, transposed to query-major; top-K     (k_combine, k_topk)
#include "hd_internal.h"
#include <algorithm>
#include <atomic>
#include <thread>

namespace hdi {
thread_local std::string g_err;
}  // namespace hdi

static int64_t ctx_bytes(const hd_ctx *c) {
    const DevBuf *all[] = {&c->rowptr, &c->col, &c->val, &c->U, &c->Ub, &c->UbT, &c->lam, &c->Usr, &c->Usc,
                           &c->Usv, &c->Ustp, &c->Ustr, &c->Ustv, &c->gfil, &c->V,
                           &c->Vb, &c->X, &c->R, &c->P, &c->Q, &c->Z, &c->Cpart, &c->Cl, &c->Cs,
                           &c->ClT, &c->CsT, &c->PT, &c->part, &c->scal, &c->xbuf, &c->sim, &c->ybuf,
                           &c->topk, &c->err, &c->qsplit, &c->Dg, &c->ymask, &c->uscale, &c->vscale, &c->pbar,
                     &c->cut, &c->pre, &c->Vsm, &c->Usm, &c->tsx};
    int64_t s = 0;
    for (const DevBuf *b : all) s += (int64_t)b->bytes;
    return s;
}

static void drop_eigs(hd_ctx *c);

// f(a, b) over [0, n) in blocks of `grain` rows on up to 16 host threads
// (each row handled by exactly one thread).
template <class F>
static void host_parallel_rows(int64_t n, int64_t grain, F f) {
    const unsigned hw = std::thread::hardware_concurrency();
    const int64_t blocks = (n + grain - 1) / grain;
    const int nt = (int)std::min<int64_t>(blocks, std::min<unsigned>(hw ? hw : 1, 16u));
    if (nt <= 1) {
        f((int64_t)0, n);
        return;
    }
    std::atomic<int64_t> next{0};
    auto work = [&] {
        for (int64_t b; (b = next.fetch_add(1)) < blocks;) f(b * grain, std::min(n, (b + 1) * grain));
    };
    std::vector<std::thread> th;
    for (int t = 1; t < nt; ++t) th.emplace_back(work);
    work();
    for (auto &t : th) t.join();
}

extern "C" {

const char *hd_last_error(void) { return g_err.c_str(); }

int hd_create(int device, hd_ctx **out) {
    g_err.clear();
    if (!out) return fail(HD_EINVAL, "hd_create: out is NULL");
    *out = nullptr;
    int count = 0;
    HIP_TRY(hipGetDeviceCount(&count));
    if (device < 0 || device >= count)
        return fail(HD_EINVAL, "hd_create: device %d not in [0, %d)", device, count);
    HIP_TRY(hipSetDevice(device));
    {
        const int e = noalloc_init(device);
        if (e != HD_OK) return e;
    }
    hd_ctx *c = new (std::nothrow) hd_ctx();
    if (!c) return fail(HD_ENOMEM, "hd_create: out of host memory");
    c->device = device;
    void *hp = nullptr;
    hipError_t e = hipHostMalloc(&hp, 256 * sizeof(int32_t), hipHostMallocDefault);
    if (e != hipSuccess) {
        delete c;
        return fail(HD_ENOMEM, "hd_create: hipHostMalloc: %s", hipGetErrorString(e));
    }
    c->h_pinned = reinterpret_cast<int32_t *>(hp);
    for (int k = 0; k < 2; ++k) {
        e = hipEventCreateWithFlags(&c->iter_ev[k], hipEventDisableTiming);
        if (e != hipSuccess) {
            hd_destroy(c);
            return fail(HD_EDEVICE, "hd_create: hipEventCreate: %s", hipGetErrorString(e));
        }
    }
    *out = c;
    return HD_OK;
}

void hd_destroy(hd_ctx *c) {
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipDeviceSynchronize();
    DevBuf *all[] = {&c->rowptr, &c->col, &c->val, &c->U, &c->Ub, &c->UbT, &c->lam, &c->Usr, &c->Usc,
                           &c->Usv, &c->Ustp, &c->Ustr, &c->Ustv, &c->gfil, &c->V,
                     &c->Vb, &c->X, &c->R, &c->P, &c->Q, &c->Z, &c->Cpart, &c->Cl, &c->Cs,
                     &c->ClT, &c->CsT, &c->PT, &c->part, &c->scal, &c->xbuf, &c->sim, &c->ybuf,
                     &c->topk, &c->err, &c->qsplit, &c->Dg, &c->ymask, &c->uscale, &c->vscale, &c->pbar,
                     &c->cut, &c->pre, &c->Vsm, &c->Usm, &c->tsx};
    for (DevBuf *b : all) b->release();
    if (c->h_pinned) (void)hipHostFree(c->h_pinned);
    for (hipEvent_t e : c->iter_ev)
        if (e) (void)hipEventDestroy(e);
    c->timing.destroy();
    delete c;
}

int64_t hd_device_bytes(const hd_ctx *c) { return c ? ctx_bytes(c) : 0; }

int hd_set_persistent(hd_ctx *c, int32_t mode, int64_t spin_limit) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_set_persistent: NULL context");
    if (mode < 0 || mode > 2) return fail(HD_EINVAL, "hd_set_persistent: mode %d not in {0, 1, 2}", mode);
    if (spin_limit < 0) return fail(HD_EINVAL, "hd_set_persistent: spin_limit < 0");
    c->persist_mode = mode;
    c->persist_spin = spin_limit > 0 ? (long long)spin_limit : (1LL << 24);
    return HD_OK;
}

int hd_timing_enable(hd_ctx *c, int enable) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_timing_enable: NULL context");
    c->timing.reset();
    c->timing.on = enable != 0;
    c->timing.mask = ~0u;
    return HD_OK;
}

int hd_timing_enable_kinds(hd_ctx *c, uint32_t kind_mask) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_timing_enable_kinds: NULL context");
    c->timing.reset();
    c->timing.on = kind_mask != 0;
    c->timing.mask = kind_mask;
    return HD_OK;
}

int hd_timing_kinds(void) { return K_NKINDS; }

const char *hd_timing_name(int kind) {
    return kind >= 0 && kind < K_NKINDS ? kKindNames[kind] : nullptr;
}

int hd_timing_get(const hd_ctx *c, int kind, double *total_ms, int64_t *launches) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_timing_get: NULL context");
    if (kind < 0 || kind >= K_NKINDS) return fail(HD_EINVAL, "hd_timing_get: kind %d out of range", kind);
    if (total_ms) *total_ms = c->timing.total_ms[kind];
    if (launches) *launches = c->timing.count[kind];
    return HD_OK;
}

int hd_load_graph(hd_ctx *c, int64_t n, int64_t nnz, const int64_t *rowptr, const int32_t *col,
                  const float *val, uint32_t flags) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_load_graph: NULL context");
    if (n <= 0 || n >= (int64_t)1 << 31) return fail(HD_EINVAL, "hd_load_graph: n=%lld out of range", (long long)n);
    if (nnz < 0) return fail(HD_EINVAL, "hd_load_graph: nnz < 0");
    if (!rowptr || (nnz > 0 && (!col || !val))) return fail(HD_EINVAL, "hd_load_graph: NULL array");
    if (flags & ~(HD_GRAPH_NORMALIZE | HD_GRAPH_CHECK_SYMMETRY))
        return fail(HD_EINVAL, "hd_load_graph: unknown flags 0x%x", flags);
    if (rowptr[0] != 0 || rowptr[n] != nnz)
        return fail(HD_EINVAL, "hd_load_graph: rowptr must start at 0 and end at nnz");
    for (int64_t i = 0; i < n; ++i) {
        const int64_t s = rowptr[i], e = rowptr[i + 1];
        if (e < s) return fail(HD_EINVAL, "hd_load_graph: rowptr decreases at row %lld", (long long)i);
        for (int64_t k = s; k < e; ++k) {
            const int32_t j = col[k];
            if (j < 0 || j >= n) return fail(HD_EINVAL, "hd_load_graph: column %d out of range in row %lld", j, (long long)i);
            if (j == i) return fail(HD_EINVAL, "hd_load_graph: diagonal entry in row %lld", (long long)i);
            if (k > s && col[k - 1] >= j)
                return fail(HD_EINVAL, "hd_load_graph: columns not strictly increasing in row %lld", (long long)i);
            if (!(val[k] >= 0.f) || !std::isfinite(val[k]))
                return fail(HD_EINVAL, "hd_load_graph: negative or non-finite value in row %lld", (long long)i);
        }
    }
    if (flags & HD_GRAPH_CHECK_SYMMETRY) {
        for (int64_t i = 0; i < n; ++i) {
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) {
                const int32_t j = col[k];
                // binary search for i in row j
                int64_t lo = rowptr[j], hi = rowptr[j + 1];
                while (lo < hi) {
                    int64_t mid = (lo + hi) / 2;
                    if (col[mid] < i) lo = mid + 1; else hi = mid;
                }
                if (lo >= rowptr[j + 1] || col[lo] != i || val[lo] != val[k])
                    return fail(HD_EINVAL, "hd_load_graph: matrix not symmetric at (%lld, %d)", (long long)i, j);
            }
        }
    }
    std::vector<float> sv;
    const float *vals = val;
    if (flags & HD_GRAPH_NORMALIZE) {
        // Section 3: S = D^-1/2 W D^-1/2, D = diag(W 1), in double precision;
        // the two scales are multiplied first so S stays exactly symmetric.
        std::vector<double> dinv((size_t)n);
        for (int64_t i = 0; i < n; ++i) {
            double deg = 0.0;
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k) deg += val[k];
            dinv[(size_t)i] = deg > 0.0 ? 1.0 / std::sqrt(deg) : 0.0;
        }
        sv.resize((size_t)nnz);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t k = rowptr[i]; k < rowptr[i + 1]; ++k)
                sv[(size_t)k] = (float)((double)val[k] * (dinv[(size_t)i] * dinv[(size_t)col[k]]));
        vals = sv.data();
    }
    HIP_TRY(hipSetDevice(c->device));
    if (c->n != n) {
        drop_eigs(c);
        c->V.release();
        c->Vb.release();
        c->vscale.release();
        c->d = c->ldv = 0;
        c->v_dtype = HD_F32;
    }
    std::vector<int32_t> cuts((size_t)n * 8);
    hd::build_band_cuts(n, rowptr, col, cuts.data());
    c->n = c->nnz = 0;  // nothing loaded until every copy has succeeded
    HIP_TRY(c->rowptr.ensure((size_t)(n + 1) * sizeof(int64_t)));
    HIP_TRY(c->col.ensure((size_t)(nnz > 0 ? nnz : 1) * sizeof(int32_t)));
    HIP_TRY(c->val.ensure((size_t)(nnz > 0 ? nnz : 1) * sizeof(float)));
    HIP_TRY(c->cut.ensure(cuts.size() * sizeof(int32_t)));
    HIP_TRY(hipMemcpy(c->rowptr.p, rowptr, (size_t)(n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->cut.p, cuts.data(), cuts.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    if (nnz > 0) {
        HIP_TRY(hipMemcpy(c->col.p, col, (size_t)nnz * sizeof(int32_t), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->val.p, vals, (size_t)nnz * sizeof(float), hipMemcpyHostToDevice));
    }
    c->n = n;
    c->nnz = nnz;
    return HD_OK;
}

// Drop every form of the loaded eigenpairs: afterwards the context holds
// none (r = 0), so no query can reach a released U1 buffer.
static void drop_eigs(hd_ctx *c) {
    for (DevBuf *b : {&c->U, &c->Ub, &c->UbT, &c->Usr, &c->Usc, &c->Usv, &c->Ustp, &c->Ustr, &c->Ustv, &c->lam,
                      &c->uscale, &c->Usm})
        b->release();
    c->usm_lo_off = 0;
    c->u_dtype = HD_F32;
    c->r = c->rp = 0;
    c->ldut = 0;
    c->us_nnz = 0;
    c->lam_host.clear();
}

// Upload FP8 E4M3 codes of U1 (n x r row-major) and their per-component
// scales: the codes in fragment order item-major (n16 x rp bytes) and
// component-major (rp x ldut bytes), padding zero, padding scales 1.
static int upload_eigs_fp8(hd_ctx *c, int r, int rp, const uint8_t *codes, const float *scales) {
    const int64_t n = c->n, ldut = (n + 63) / 64 * 64, n16 = (n + 15) / 16 * 16;
    std::vector<uint8_t> im((size_t)n16 * rp, 0), cm((size_t)rp * ldut, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < r; ++k) {
            const uint8_t q = codes[(size_t)i * r + k];
            im[hd::frag_offset(i, k, rp / 32)] = q;
            cm[hd::frag_offset(k, i, ldut / 32)] = q;
        }
    std::vector<float> sc((size_t)rp, 1.0f);
    for (int k = 0; k < r; ++k) sc[(size_t)k] = scales[k];
    HIP_TRY(c->Ub.ensure(im.size()));
    HIP_TRY(c->UbT.ensure(cm.size()));
    HIP_TRY(c->uscale.ensure(sc.size() * sizeof(float)));
    HIP_TRY(hipMemcpy(c->Ub.p, im.data(), im.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->UbT.p, cm.data(), cm.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->uscale.p, sc.data(), sc.size() * sizeof(float), hipMemcpyHostToDevice));
    c->ldut = ldut;
    return HD_OK;
}

static int load_eigs_dense(hd_ctx *c, int r, int rp, const float *U, int dtype);
static int upload_descriptors(hd_ctx *c, int d, int ldv, const float *V, int dtype);

// The one-pass top-K's row samples (hd::topk_sample) of the stored matrix-core
// forms, built on the device from the stored copies: the sampled item-major
// U1 rows (each term) and the sampled descriptors (with their fp8 row
// scales). None for fp32 storage or n < hd::kTopkFuseMin.
static int build_usample(hd_ctx *c) {
    c->Usm.release();
    c->usm_lo_off = 0;
    if (c->n < hd::kTopkFuseMin || !c->u_mfma() || c->rp == 0) return HD_OK;
    int64_t st, m;
    hd::topk_sample(c->n, &st, &m);
    const int eb = c->u_fp8() ? 1 : 2, terms = c->u_dtype == HD_BF16X2 ? 2 : 1;
    const size_t per = (size_t)((m + 15) / 16 * 16) * c->rp * eb, per_src = (size_t)((c->n + 15) / 16 * 16) * c->rp * eb;
    HIP_TRY(c->Usm.ensure(per * terms));
    for (int t = 0; t < terms; ++t)
        HIP_TRY(hd::launch_sample_frag(m, st, c->rp, c->Ub.as<char>() + t * per_src, c->Usm.as<char>() + t * per, eb,
                                       nullptr));
    HIP_TRY(hipStreamSynchronize(nullptr));
    c->usm_lo_off = per;
    return HD_OK;
}

static int build_vsample(hd_ctx *c) {
    c->Vsm.release();
    c->vsm_scale_off = 0;
    if (c->n < hd::kTopkFuseMin || c->v_dtype == HD_F32) return HD_OK;
    int64_t st, m;
    hd::topk_sample(c->n, &st, &m);
    const bool fp8 = c->v_dtype == HD_FP8_E4M3;
    const int eb = fp8 ? 1 : 2;
    const size_t codes = ((size_t)((m + 15) / 16 * 16) * c->ldv * eb + 255) / 256 * 256;
    HIP_TRY(c->Vsm.ensure(codes + (fp8 ? (size_t)m * sizeof(float) : 0)));
    HIP_TRY(hd::launch_sample_frag(m, st, c->ldv, c->Vb.p, c->Vsm.p, eb, nullptr));
    if (fp8)
        HIP_TRY(hd::launch_sample_rows(m, st, 1, c->vscale.as<float>(),
                                       reinterpret_cast<float *>(c->Vsm.as<char>() + codes), nullptr));
    HIP_TRY(hipStreamSynchronize(nullptr));
    c->vsm_scale_off = codes;
    return HD_OK;
}

// The common tail of the eigenpair loaders: eigenvalues and the form.
static int finish_eigs(hd_ctx *c, int r, int rp, const double *lambda, int dtype) {
    std::vector<double> lam((size_t)rp, 0.0);
    for (int k = 0; k < r; ++k) lam[(size_t)k] = lambda[k];
    HIP_TRY(c->lam.ensure(lam.size() * sizeof(double)));
    HIP_TRY(hipMemcpy(c->lam.p, lam.data(), lam.size() * sizeof(double), hipMemcpyHostToDevice));
    c->lam_host = lam;
    c->r = r;
    c->rp = rp;
    c->u_dtype = dtype;
    return build_usample(c);
}

int hd_load_eigs_fp8(hd_ctx *c, int32_t r, const uint8_t *codes, const float *col_scale, const double *lambda) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_load_eigs_fp8: NULL context");
    if (c->n == 0) return fail(HD_ESTATE, "hd_load_eigs_fp8: no graph loaded");
    if (r < 1 || r > c->n) return fail(HD_EINVAL, "hd_load_eigs_fp8: r=%d not in [1, n]", r);
    if (!codes || !col_scale || !lambda) return fail(HD_EINVAL, "hd_load_eigs_fp8: NULL array");
    for (int k = 0; k < r; ++k) {
        if (!(std::fabs(lambda[k]) <= 1.0 + 1e-6))
            return fail(HD_EINVAL, "hd_load_eigs_fp8: lambda[%d]=%g outside [-1, 1]", k, lambda[k]);
        if (!(col_scale[k] > 0.0f) || !std::isfinite(col_scale[k]))
            return fail(HD_EINVAL, "hd_load_eigs_fp8: col_scale[%d] not positive and finite", k);
    }
    const int64_t n = c->n;
    for (size_t t = 0; t < (size_t)n * r; ++t)
        if (fp8_e4m3_is_nan(codes[t])) return fail(HD_EINVAL, "hd_load_eigs_fp8: NaN code at %zu", t);
    HIP_TRY(hipSetDevice(c->device));
    drop_eigs(c);
    const int rp = (r + 31) / 32 * 32;
    int e = upload_eigs_fp8(c, r, rp, codes, col_scale);
    if (e == HD_OK) e = finish_eigs(c, r, rp, lambda, HD_FP8_E4M3);
    if (e != HD_OK) drop_eigs(c);
    return e;
}

int hd_load_eigs(hd_ctx *c, int32_t r, const float *U, const double *lambda, int32_t dtype) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_load_eigs: NULL context");
    if (c->n == 0) return fail(HD_ESTATE, "hd_load_eigs: no graph loaded");
    if (r < 0 || r > c->n) return fail(HD_EINVAL, "hd_load_eigs: r=%d not in [0, n]", r);
    if (dtype != HD_F32 && dtype != HD_BF16 && dtype != HD_BF16X2 && dtype != HD_FP8_E4M3)
        return fail(HD_EINVAL, "hd_load_eigs: dtype %d not supported", dtype);
    const int64_t n = c->n;
    // every check comes before the context is touched: a rejected call leaves
    // the loaded eigenpairs as they were
    if (r > 0) {
        if (!U || !lambda) return fail(HD_EINVAL, "hd_load_eigs: NULL array");
        for (int k = 0; k < r; ++k)
            // the spectrum of S lies in [-1, 1]; allow eigensolver rounding
            if (!(std::fabs(lambda[k]) <= 1.0 + 1e-6))
                return fail(HD_EINVAL, "hd_load_eigs: lambda[%d]=%g outside [-1, 1]", k, lambda[k]);
        for (int64_t i = 0; i < n; ++i)
            for (int k = 0; k < r; ++k)
                if (!std::isfinite(U[(size_t)i * r + k]))
                    return fail(HD_EINVAL, "hd_load_eigs: non-finite U at row %lld", (long long)i);
    }
    HIP_TRY(hipSetDevice(c->device));
    // from here on a failure (allocation, copy) leaves no eigenpairs loaded
    drop_eigs(c);
    if (r == 0) return HD_OK;
    const int rp = (r + 31) / 32 * 32;
    const int e = load_eigs_dense(c, r, rp, U, dtype);
    if (e != HD_OK) {
        drop_eigs(c);
        return e;
    }
    const int f = finish_eigs(c, r, rp, lambda, dtype);
    if (f != HD_OK) drop_eigs(c);
    return f;
}

// The device copies of a dense U1 (n x r fp32 host, validated) in the form
// `dtype`; on failure the caller drops what was allocated.
static int load_eigs_dense(hd_ctx *c, int r, int rp, const float *U, int dtype) {
    const int64_t n = c->n;
    if (dtype == HD_FP8_E4M3) {
        std::vector<uint8_t> codes((size_t)n * r);
        std::vector<float> sc((size_t)r);
        fp8_quantize(n, r, U, true, codes.data(), sc.data());
        return upload_eigs_fp8(c, r, rp, codes.data(), sc.data());
    }
    if (dtype == HD_F32) {
        std::vector<float> host((size_t)n * rp, 0.f);
        host_parallel_rows(n, 4096, [&](int64_t a, int64_t b) {
            for (int64_t i = a; i < b; ++i)
                std::memcpy(host.data() + (size_t)i * rp, U + (size_t)i * r, (size_t)r * sizeof(float));
        });
        HIP_TRY(c->U.ensure(host.size() * sizeof(float)));
        HIP_TRY(hipMemcpy(c->U.p, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice));
    } else {
        // hi terms first; the two-term form appends the lo terms (same
        // layout). Both copies are in fragment order: item-major over
        // n16 x rp (rows padded to 16), component-major over rp x ldut.
        const int64_t ldut = (n + 63) / 64 * 64, n16 = (n + 15) / 16 * 16;
        const int terms = dtype == HD_BF16X2 ? 2 : 1;
        const size_t imn = (size_t)n16 * rp, cmn = (size_t)rp * ldut;
        std::vector<uint16_t> im(imn * terms, 0), cm(cmn * terms, 0);
        // blocks of 64 items: whole 16-row tiles of both layouts per thread
        host_parallel_rows(n, 64, [&](int64_t a, int64_t b) {
            for (int64_t i = a; i < b; ++i)
                for (int k = 0; k < r; ++k) {
                    const float u = U[(size_t)i * r + k];
                    const uint16_t h = bf16_rne_host(u);
                    const size_t oi = hd::frag_offset(i, k, rp / 32), oc = hd::frag_offset(k, i, ldut / 32);
                    im[oi] = h;
                    cm[oc] = h;
                    if (terms == 2) {
                        float hf;
                        const uint32_t hb = (uint32_t)h << 16;
                        std::memcpy(&hf, &hb, sizeof(hf));
                        const uint16_t l = bf16_rne_host(u - hf);
                        im[imn + oi] = l;
                        cm[cmn + oc] = l;
                    }
                }
        });
        HIP_TRY(c->Ub.ensure(im.size() * sizeof(uint16_t)));
        HIP_TRY(c->UbT.ensure(cm.size() * sizeof(uint16_t)));
        HIP_TRY(hipMemcpy(c->Ub.p, im.data(), im.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->UbT.p, cm.data(), cm.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
        c->ldut = ldut;
    }
    return HD_OK;
}

static int load_eigs_sparse(hd_ctx *c, int32_t r, int64_t nnz, const int64_t *rowptr, const int32_t *col,
                            const float *val, const double *lambda);

int hd_load_eigs_sparse(hd_ctx *c, int32_t r, int64_t nnz, const int64_t *rowptr, const int32_t *col,
                        const float *val, const double *lambda) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_load_eigs_sparse: NULL context");
    if (c->n == 0) return fail(HD_ESTATE, "hd_load_eigs_sparse: no graph loaded");
    const int64_t n = c->n;
    if (r < 1 || r > n) return fail(HD_EINVAL, "hd_load_eigs_sparse: r=%d not in [1, n]", r);
    if (nnz < 0 || !rowptr || !lambda || (nnz > 0 && (!col || !val)))
        return fail(HD_EINVAL, "hd_load_eigs_sparse: NULL array or nnz < 0");
    if (rowptr[0] != 0 || rowptr[n] != nnz) return fail(HD_EINVAL, "hd_load_eigs_sparse: rowptr must run from 0 to nnz");
    for (int64_t i = 0; i < n; ++i) {
        if (rowptr[i + 1] < rowptr[i]) return fail(HD_EINVAL, "hd_load_eigs_sparse: rowptr decreases at row %lld", (long long)i);
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
            if (col[e] < 0 || col[e] >= r || (e > rowptr[i] && col[e] <= col[e - 1]))
                return fail(HD_EINVAL, "hd_load_eigs_sparse: row %lld: component ids out of range or not increasing", (long long)i);
            if (!std::isfinite(val[e])) return fail(HD_EINVAL, "hd_load_eigs_sparse: non-finite value in row %lld", (long long)i);
        }
    }
    for (int k = 0; k < r; ++k)
        if (!(std::fabs(lambda[k]) <= 1.0 + 1e-6))
            return fail(HD_EINVAL, "hd_load_eigs_sparse: lambda[%d]=%g outside [-1, 1]", k, lambda[k]);
    HIP_TRY(hipSetDevice(c->device));
    drop_eigs(c);
    const int e = load_eigs_sparse(c, r, nnz, rowptr, col, val, lambda);
    if (e != HD_OK) drop_eigs(c);
    return e;
}

// The device copies of a validated sparsified U1 (by item and by component).
static int load_eigs_sparse(hd_ctx *c, int32_t r, int64_t nnz, const int64_t *rowptr, const int32_t *col,
                            const float *val, const double *lambda) {
    const int64_t n = c->n;
    const int rp = (r + 31) / 32 * 32;
    // by-component copy: counting sort of the entries by component
    std::vector<int64_t> cptr((size_t)rp + 1, 0);
    for (int64_t e = 0; e < nnz; ++e) ++cptr[(size_t)col[e] + 1];
    for (int k = 0; k < rp; ++k) cptr[(size_t)k + 1] += cptr[(size_t)k];
    std::vector<int32_t> crow((size_t)(nnz > 0 ? nnz : 1));
    std::vector<float> cval((size_t)(nnz > 0 ? nnz : 1));
    {
        std::vector<int64_t> fill(cptr.begin(), cptr.end() - 1);
        for (int64_t i = 0; i < n; ++i)
            for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) {
                const int64_t p = fill[(size_t)col[e]]++;
                crow[(size_t)p] = (int32_t)i;
                cval[(size_t)p] = val[e];
            }
    }
    const size_t nz = (size_t)(nnz > 0 ? nnz : 1);
    HIP_TRY(c->Usr.ensure((size_t)(n + 1) * sizeof(int64_t)));
    HIP_TRY(c->Usc.ensure(nz * sizeof(int32_t)));
    HIP_TRY(c->Usv.ensure(nz * sizeof(float)));
    HIP_TRY(c->Ustp.ensure(cptr.size() * sizeof(int64_t)));
    HIP_TRY(c->Ustr.ensure(nz * sizeof(int32_t)));
    HIP_TRY(c->Ustv.ensure(nz * sizeof(float)));
    HIP_TRY(hipMemcpy(c->Usr.p, rowptr, (size_t)(n + 1) * sizeof(int64_t), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->Ustp.p, cptr.data(), cptr.size() * sizeof(int64_t), hipMemcpyHostToDevice));
    if (nnz > 0) {
        HIP_TRY(hipMemcpy(c->Usc.p, col, (size_t)nnz * sizeof(int32_t), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->Usv.p, val, (size_t)nnz * sizeof(float), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->Ustr.p, crow.data(), (size_t)nnz * sizeof(int32_t), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(c->Ustv.p, cval.data(), (size_t)nnz * sizeof(float), hipMemcpyHostToDevice));
    }
    c->us_nnz = nnz;
    return finish_eigs(c, r, rp, lambda, HD_SPARSE_F32);
}

// Upload FP8 E4M3 descriptor codes (n x d row-major) in fragment order over
// n16 x ldv bytes (zero padded) and one scale per row.
static int upload_descriptors_fp8(hd_ctx *c, int d, int ldv, const uint8_t *codes, const float *row_scale) {
    const int64_t n = c->n, n16 = (n + 15) / 16 * 16;
    std::vector<uint8_t> host((size_t)n16 * ldv, 0);
    for (int64_t i = 0; i < n; ++i)
        for (int t = 0; t < d; ++t) host[hd::frag_offset(i, t, ldv / 32)] = codes[(size_t)i * d + t];
    HIP_TRY(c->Vb.ensure(host.size()));
    HIP_TRY(c->vscale.ensure((size_t)n * sizeof(float)));
    HIP_TRY(hipMemcpy(c->Vb.p, host.data(), host.size(), hipMemcpyHostToDevice));
    HIP_TRY(hipMemcpy(c->vscale.p, row_scale, (size_t)n * sizeof(float), hipMemcpyHostToDevice));
    return HD_OK;
}

static void drop_descriptors(hd_ctx *c) {
    c->V.release();
    c->Vb.release();
    c->vscale.release();
    c->Vsm.release();
    c->vsm_scale_off = 0;
    c->d = c->ldv = 0;
    c->v_dtype = HD_F32;
}

int hd_load_descriptors_fp8(hd_ctx *c, int32_t d, const uint8_t *codes, const float *row_scale) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_load_descriptors_fp8: NULL context");
    if (c->n == 0) return fail(HD_ESTATE, "hd_load_descriptors_fp8: no graph loaded");
    if (d <= 0 || !codes || !row_scale) return fail(HD_EINVAL, "hd_load_descriptors_fp8: bad d or NULL array");
    const int64_t n = c->n;
    for (int64_t i = 0; i < n; ++i)
        if (!(row_scale[i] > 0.0f) || !std::isfinite(row_scale[i]))
            return fail(HD_EINVAL, "hd_load_descriptors_fp8: row_scale[%lld] not positive and finite", (long long)i);
    for (size_t t = 0; t < (size_t)n * d; ++t)
        if (fp8_e4m3_is_nan(codes[t])) return fail(HD_EINVAL, "hd_load_descriptors_fp8: NaN code at %zu", t);
    HIP_TRY(hipSetDevice(c->device));
    drop_descriptors(c);
    const int ldv = (d + 31) / 32 * 32;
    const int e = upload_descriptors_fp8(c, d, ldv, codes, row_scale);
    if (e != HD_OK) {
        drop_descriptors(c);
        return e;
    }
    c->d = d;
    c->ldv = ldv;
    c->v_dtype = HD_FP8_E4M3;
    const int f = build_vsample(c);
    if (f != HD_OK) drop_descriptors(c);
    return f;
}

int hd_load_descriptors(hd_ctx *c, int32_t d, const float *V, int32_t dtype) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_load_descriptors: NULL context");
    if (c->n == 0) return fail(HD_ESTATE, "hd_load_descriptors: no graph loaded");
    if (d <= 0 || !V) return fail(HD_EINVAL, "hd_load_descriptors: bad d or NULL V");
    if (dtype != HD_F32 && dtype != HD_BF16 && dtype != HD_FP8_E4M3)
        return fail(HD_EINVAL, "hd_load_descriptors: dtype %d not supported", dtype);
    const int ldv = (d + 31) / 32 * 32;
    const int64_t n = c->n;
    for (int64_t i = 0; i < n; ++i)
        for (int t = 0; t < d; ++t)
            if (!std::isfinite(V[(size_t)i * d + t]))
                return fail(HD_EINVAL, "hd_load_descriptors: non-finite V at row %lld", (long long)i);
    HIP_TRY(hipSetDevice(c->device));
    drop_descriptors(c);
    int e = HD_OK;
    if (dtype == HD_FP8_E4M3) {
        std::vector<uint8_t> codes((size_t)n * d);
        std::vector<float> sc((size_t)n);
        fp8_quantize(n, d, V, false, codes.data(), sc.data());
        e = upload_descriptors_fp8(c, d, ldv, codes.data(), sc.data());
    } else {
        e = upload_descriptors(c, d, ldv, V, dtype);
    }
    if (e != HD_OK) {
        drop_descriptors(c);
        return e;
    }
    c->d = d;
    c->ldv = ldv;
    c->v_dtype = dtype;
    const int f = build_vsample(c);
    if (f != HD_OK) drop_descriptors(c);
    return f;
}

// fp32 (n x ldv, zero padded) or bfloat16 (fragment order over n16 x ldv)
// device copies of validated descriptors.
static int upload_descriptors(hd_ctx *c, int d, int ldv, const float *V, int dtype) {
    const int64_t n = c->n;
    if (dtype == HD_F32) {
        std::vector<float> host((size_t)n * ldv, 0.f);
        for (int64_t i = 0; i < n; ++i)
            std::memcpy(host.data() + (size_t)i * ldv, V + (size_t)i * d, (size_t)d * sizeof(float));
        HIP_TRY(c->V.ensure(host.size() * sizeof(float)));
        HIP_TRY(hipMemcpy(c->V.p, host.data(), host.size() * sizeof(float), hipMemcpyHostToDevice));
    } else {
        // fragment order over n16 x ldv (rows padded to 16), the operand
        // order of the similarity kernel's matrix-core loads
        const int64_t n16 = (n + 15) / 16 * 16;
        std::vector<uint16_t> host((size_t)n16 * ldv, 0);
        for (int64_t i = 0; i < n; ++i)
            for (int t = 0; t < d; ++t)
                host[hd::frag_offset(i, t, ldv / 32)] = bf16_rne_host(V[(size_t)i * d + t]);
        HIP_TRY(c->Vb.ensure(host.size() * sizeof(uint16_t)));
        HIP_TRY(hipMemcpy(c->Vb.p, host.data(), host.size() * sizeof(uint16_t), hipMemcpyHostToDevice));
    }
    return HD_OK;
}

int hd_rank(hd_ctx *c, int32_t B, int64_t n, const float *x, int64_t ldx, int32_t K,
            int32_t *ids_out, float *scores_out, void *stream) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_rank: NULL context");
    if (B < 1 || n < 1 || ldx < n || !x) return fail(HD_EINVAL, "hd_rank: bad B, n, ldx or x");
    if (K < 1 || K > n || K > hd::kTopkMax)
        return fail(HD_EINVAL, "hd_rank: K=%d not in [1, min(n, %d)]", K, hd::kTopkMax);
    if (!ids_out && !scores_out) return HD_OK;
    HIP_TRY(hipSetDevice(c->device));
    HIP_TRY(c->topk.ensure(hd::topk_scratch_bytes(B, n, K)));
    HIP_TRY(hd::launch_topk(B, n, x, ldx, K, c->topk.p, ids_out, scores_out, 0, (hipStream_t)stream));
    return HD_OK;
}

}  // extern "C"

// Bytes of the one-pass top-K's per-batch sample buffer (c->tsx): the B x m
// sample scores (rows padded to 64) and m sampled rows of x^t at the widest
// solver width; one size for both selections of a query, so the second
// never reallocates the buffer under the first.
static size_t onepass_sample_bytes(int B, int64_t m) {
    return ((size_t)B * (size_t)((m + 63) / 64 * 64) + (size_t)m * 1024) * sizeof(float);
}

// Step 1 (Section 3; Section 6.1): the observation vectors y of B queries from
// their descriptors (similarities to every item, the k_y largest, cubed), or
// the given sparse y copied to the optional outputs. *yi / *yv receive the
// device arrays of y the later steps read.
static int queue_y(hd_ctx *c, int32_t B, const float *q_desc, const int32_t *y_ids, const float *y_val, int ky,
                   int32_t *y_ids_out, float *y_val_out, hipStream_t s, const int32_t **yi, const float **yv) {
    const int64_t n = c->n;
    if (q_desc) {
        const int64_t lds = (n + 63) / 64 * 64;
        HIP_TRY(c->sim.ensure((size_t)B * lds * sizeof(float)));
        HIP_TRY(c->topk.ensure(hd::topk_scratch_bytes(B, n, ky)));
        int32_t *oi = y_ids_out;
        float *ov = y_val_out;
        if (!oi || !ov) {
            HIP_TRY(c->ybuf.ensure((size_t)B * ky * (sizeof(int32_t) + sizeof(float))));
            oi = c->ybuf.as<int32_t>();
            ov = reinterpret_cast<float *>(oi + (size_t)B * ky);
        }
        if (c->v_dtype != HD_F32) {
            HIP_TRY(c->qsplit.ensure((size_t)2 * hd::sim_qsplit_rows(B) * c->ldv * sizeof(uint16_t)));
        }
        uint16_t *qs = c->qsplit.as<uint16_t>();
        if (c->v_dtype != HD_F32 && c->onepass_y()) {
            // one-pass top-k_y: thresholds from the sampled items'
            // similarities, then the similarity kernel offers every value to
            // the lists without writing sim; sim is written only if some row
            // needs the exact fallback
            int64_t st, m;
            hd::topk_sample(n, &st, &m);
            const int64_t lss = (m + 63) / 64 * 64;
            HIP_TRY(c->tsx.ensure(onepass_sample_bytes(B, m)));
            const hd::TopkLists tl = hd::topk_lists(c->topk.p, B, n);
            const int32_t *gate = hd::topk_fallback_gate(c->topk.p, B, n);
            LAUNCH(K_TOPK_Y, hd::launch_sim_bf16(m, B, c->d, q_desc, c->Vsm.p, c->ldv, qs, c->tsx.as<float>(), lss, s,
                                                 c->vsm_scale()));
            LAUNCH(K_TOPK_Y, hd::launch_topk_prepare(B, n, c->tsx.as<float>(), lss, 1, ky, c->topk.p, s));
            LAUNCH(K_SIM, hd::launch_sim_bf16(n, B, c->d, q_desc, c->Vb.p, c->ldv, qs, nullptr, lds, s, c->v_scale(),
                                              &tl, nullptr, false));
            LAUNCH(K_TOPK_Y, hd::launch_topk_select_lists(B, n, ky, c->topk.p, oi, ov, 1, s));
            LAUNCH(K_TOPK_Y, hd::launch_sim_bf16(n, B, c->d, q_desc, c->Vb.p, c->ldv, qs, c->sim.as<float>(), lds, s,
                                                 c->v_scale(), nullptr, gate, false));
            LAUNCH(K_TOPK_Y, hd::launch_topk_fallback(B, n, c->sim.as<float>(), lds, ky, c->topk.p, oi, ov, 1, s));
        } else {
            if (c->v_dtype != HD_F32) {
                LAUNCH(K_SIM, hd::launch_sim_bf16(n, B, c->d, q_desc, c->Vb.p, c->ldv, qs, c->sim.as<float>(), lds, s,
                                                  c->v_scale()));
            } else {
                LAUNCH(K_SIM, hd::launch_sim(n, B, c->d, q_desc, c->V.as<float>(), c->ldv, c->sim.as<float>(), lds, s));
            }
            LAUNCH(K_TOPK_Y, hd::launch_topk(B, n, c->sim.as<float>(), lds, ky, c->topk.p, oi, ov, 1, s));
        }
        *yi = oi;
        *yv = ov;
    } else {
        if (y_ids_out) HIP_TRY(hipMemcpyAsync(y_ids_out, y_ids, (size_t)B * ky * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        if (y_val_out) HIP_TRY(hipMemcpyAsync(y_val_out, y_val, (size_t)B * ky * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    return HD_OK;
}

// The persistent form of steps 2-4 for a narrow batch (queue_query checked
// the arguments and the eligibility): W = the batch width rounded up to a
// power of two; plain CG (rk = 0) or fp32 U1. Set-up kernels (y scatter, y^T
// y, spectral coefficients), one persistent kernel for every CG iteration,
// the narrow combine and the ranking.
static int queue_persist(hd_ctx *c, int32_t B, const float *q_desc, const int32_t *y_ids, const float *y_val,
                         const hd_query_opts *o, int r_use, int rk, int W, int32_t *rank_ids, float *rank_scores,
                         float *x_out, int32_t *y_ids_out, float *y_val_out, hipStream_t s, bool graph,
                         int *last_iter_out) {
    const int64_t n = c->n;
    const int ky = o->k_y;
    const int G = hd::persist_grid(W, rk, n);
    if (G < 1) return fail(HD_EDEVICE, "hd_query_batch: no co-resident grid for the persistent CG (width %d)", W);
    const size_t vec = (size_t)n * W * sizeof(float);
    HIP_TRY(c->X.ensure(vec));
    HIP_TRY(c->R.ensure(vec));
    HIP_TRY(c->P.ensure(vec));
    HIP_TRY(c->Q.ensure(vec));
    if (rk > 0) {
        HIP_TRY(c->Cl.ensure((size_t)rk * W * sizeof(float)));
        HIP_TRY(c->Cs.ensure((size_t)rk * W * sizeof(float)));
        HIP_TRY(c->Cpart.ensure((size_t)G * rk * W * sizeof(float)));
    }
    HIP_TRY(c->part.ensure((size_t)(2 * G + 1) * W * sizeof(double)));
    HIP_TRY(c->scal.ensure((size_t)W * (5 * sizeof(double) + 3 * sizeof(int32_t)) + 128 * sizeof(int32_t)));
    HIP_TRY(c->err.ensure(sizeof(int32_t) * 4));
    HIP_TRY(c->pbar.ensure(sizeof(uint32_t) * 4));
    {
        char *b = c->scal.as<char>();
        hd::CgState &st = c->st;
        st.rho0 = reinterpret_cast<double *>(b); b += W * sizeof(double);
        st.rho = reinterpret_cast<double *>(b); b += W * sizeof(double);
        st.a = reinterpret_cast<double *>(b); b += W * sizeof(double);
        st.beta = reinterpret_cast<double *>(b); b += W * sizeof(double);
        st.relres = reinterpret_cast<double *>(b); b += W * sizeof(double);
        st.active = reinterpret_cast<int32_t *>(b); b += W * sizeof(int32_t);
        st.iters = reinterpret_cast<int32_t *>(b); b += W * sizeof(int32_t);
        st.status = reinterpret_cast<int32_t *>(b); b += W * sizeof(int32_t);
        st.nact_part = reinterpret_cast<int32_t *>(b);
        st.maxit = nullptr;
    }
    const hd::CgState st = c->st;
    const int32_t *yi = y_ids;
    const float *yv = y_val;
    {
        const int e = queue_y(c, B, q_desc, y_ids, y_val, ky, y_ids_out, y_val_out, s, &yi, &yv);
        if (e != HD_OK) return e;
    }
    float *X = c->X.as<float>(), *R = c->R.as<float>(), *P = c->P.as<float>(), *Q = c->Q.as<float>();
    double *gpart = c->part.as<double>(), *rpart = gpart + (size_t)G * W, *yn = rpart + (size_t)G * W;
    const size_t nv = (size_t)n * W;
    LAUNCH(K_FILL, hd::launch_fill_zero(X, nv, s));
    LAUNCH(K_FILL, hd::launch_fill_zero(R, nv, s));
    LAUNCH(K_FILL, hd::launch_fill_zero(P, nv, s));
    LAUNCH(K_FILL, hd::launch_fill_zero(reinterpret_cast<float *>(c->err.p), 2, s));
    LAUNCH(K_FILL, hd::launch_fill_zero(reinterpret_cast<float *>(c->pbar.p), 4, s));
    LAUNCH(K_SCATTER, hd::launch_scatter_y(B, ky, yi, yv, n, W, R, P, c->err.as<int32_t>(), s));
    LAUNCH(K_COLSQ, hd::launch_ynorm_part(B, ky, yi, n, W, R, yn, s));
    if (!graph) {
        HIP_TRY(hipMemcpyAsync(c->h_pinned + 200, c->err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (c->timing.on) HIP_TRY(c->timing.harvest(0));
        if (c->h_pinned[200] != 0) return fail(HD_EINVAL, "hd_query_batch: a y id is outside [0, n)");
    }
    const float *U = c->U.as<float>();
    if (rk > 0)
        LAUNCH(K_GATHER, hd::launch_gather_proj(B, ky, yi, yv, n, U, nullptr, 0, c->rp, rk, r_use, c->lam.as<double>(),
                                                o->alpha, W, c->Cs.as<float>(), c->Cl.as<float>(), s));
    c->timing.tag = 1;
    LAUNCH(K_PERSIST, hd::launch_cg_persist(W, G, n, c->rowptr.as<int64_t>(), c->col.as<int32_t>(),
                                            c->val.as<float>(), rk > 0 ? U : nullptr, c->rp, rk, r_use,
                                            c->lam.as<double>(), o->alpha, X, R, P, Q, c->Cl.as<float>(),
                                            c->Cpart.as<float>(), gpart, rpart, yn, st, B, o->max_iter, o->tol,
                                            c->pbar.as<uint32_t>(), c->persist_spin, c->err.as<int32_t>(), s));
    c->timing.tag = 0;
    LAUNCH(K_SCALAR, hd::launch_cg_final(W, st, s));
    if (!graph) {
        HIP_TRY(hipMemcpyAsync(c->h_pinned + 201, c->err.as<int32_t>() + 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (c->h_pinned[201] != 0)
            return fail(HD_EDEVICE, "hd_query_batch: a grid barrier wait of the persistent CG ran past its limit");
    }
    float *xq = x_out;
    if (!xq) {
        HIP_TRY(c->xbuf.ensure((size_t)B * n * sizeof(float)));
        xq = c->xbuf.as<float>();
    }
    if (x_out || o->top_k > 0)
        LAUNCH(K_COMBINE, hd::launch_combine_narrow(W, n, B, rk > 0 ? U : nullptr, c->rp, rk, c->Cs.as<float>(), X, xq,
                                                    n, s));
    if (o->top_k > 0 && (rank_ids || rank_scores)) {
        HIP_TRY(c->topk.ensure(hd::topk_scratch_bytes(B, n, o->top_k)));
        LAUNCH(K_TOPK_RANK, hd::launch_topk(B, n, xq, n, o->top_k, c->topk.p, rank_ids, rank_scores, 0, s));
    }
    if (last_iter_out) *last_iter_out = o->max_iter;
    return HD_OK;
}

int hdi::queue_query(hd_ctx *c, int32_t B, const float *q_desc, const int32_t *y_ids,
                     const float *y_val, const hd_query_opts *o, int32_t *rank_ids,
                     float *rank_scores, float *x_out, int32_t *y_ids_out, float *y_val_out,
                     hipStream_t s, bool graph, int *last_iter_out, const Filter *flt) {
    if (!c) return fail(HD_EINVAL, "hd_query_batch: NULL context");
    if (c->n == 0) return fail(HD_ESTATE, "hd_query_batch: no graph loaded");
    if (!o) return fail(HD_EINVAL, "hd_query_batch: NULL options");
    if (B < 1 || B > 1024) return fail(HD_EINVAL, "hd_query_batch: B=%d not in [1, 1024]", B);
    if (!(o->alpha >= 0.0 && o->alpha < 1.0)) return fail(HD_EINVAL, "hd_query_batch: alpha=%g not in [0, 1)", o->alpha);
    if (o->max_iter < 0) return fail(HD_EINVAL, "hd_query_batch: max_iter < 0");
    if (std::isnan(o->tol)) return fail(HD_EINVAL, "hd_query_batch: tol is NaN");
    const int64_t n = c->n;
    const int ky = o->k_y;
    if (ky < 1 || ky > n || ky > hd::kTopkMax) return fail(HD_EINVAL, "hd_query_batch: k_y=%d out of range", ky);
    if (o->top_k < 0 || o->top_k > n || o->top_k > hd::kTopkMax)
        return fail(HD_EINVAL, "hd_query_batch: top_k=%d out of range", o->top_k);
    const int r_use = o->rank_r < 0 ? c->r : o->rank_r;
    if (r_use > c->r) return fail(HD_ESTATE, "hd_query_batch: rank_r=%d above the %d loaded eigenpairs", r_use, c->r);
    if (q_desc) {
        if (c->d == 0) return fail(HD_ESTATE, "hd_query_batch: descriptors not loaded");
    } else if (!y_ids || !y_val) {
        return fail(HD_EINVAL, "hd_query_batch: give q_desc or both y_ids and y_val");
    }
    HIP_TRY(hipSetDevice(c->device));

    if (c->persist_mode != 0 && !flt && !c->u_sparse() && (r_use == 0 || c->u_dtype == HD_F32)) {
        int W = 1;
        while (W < B) W <<= 1;
        const int rkp = (r_use + 31) / 32 * 32;
        if (B <= (c->persist_mode == 2 ? 64 : 16) && hd::persist_width_ok(W, rkp) && hd::persist_grid(W, rkp, n) > 0)
            return queue_persist(c, B, q_desc, y_ids, y_val, o, r_use, rkp, W, rank_ids, rank_scores, x_out,
                                 y_ids_out, y_val_out, s, graph, last_iter_out);
    }

    const int ldb = pow2_at_least(B);
    const size_t vec = (size_t)n * ldb * sizeof(float);
    // the sparsified form keeps every loaded component's coefficient row (its
    // item rows may name any of them; rows past r_use stay zero)
    const bool sparse = c->u_sparse();
    const int rk = sparse ? (r_use > 0 ? c->rp : 0) : (r_use + 31) / 32 * 32;
    const hd::RowPart rp = hd::make_row_part(n);
    int64_t rc;
    const int nchunk = hd::ut_p_chunks(n, &rc);
    // Dense bfloat16 U1 in CG: the eigenvector correction follows the sparse
    // product (Q = Qs + alpha / (1 - alpha) U1 L1 U1^T P, Qs = (P - alpha S P) /
    // (1 - alpha)) and U1 C is applied inside the residual update, so Q is
    // never stored; gamma = P^T Qs + alpha / (1 - alpha) (U1^T P)^T L1 (U1^T P).
    const bool fused = rk > 0 && !sparse && c->u_mfma() && !flt;
    const int nrb = hd::uc_update_r_blocks(n);
    HIP_TRY(c->X.ensure(vec));
    HIP_TRY(c->R.ensure(vec));
    HIP_TRY(c->P.ensure(vec));
    HIP_TRY(c->Q.ensure(vec));
    if (fused) HIP_TRY(c->Dg.ensure((size_t)rk * ldb * sizeof(double)));
    if (rk > 0) {
        if (!fused) HIP_TRY(c->Z.ensure(vec));
        if (!sparse) HIP_TRY(c->Cpart.ensure((size_t)nchunk * rk * ldb * sizeof(float)));
        HIP_TRY(c->Cl.ensure((size_t)rk * ldb * sizeof(float)));
        HIP_TRY(c->Cs.ensure((size_t)rk * ldb * sizeof(float)));
        if (c->u_mfma()) {
            HIP_TRY(c->ClT.ensure((size_t)rk * ldb * 2 * sizeof(uint16_t)));
            HIP_TRY(c->CsT.ensure((size_t)rk * ldb * 2 * sizeof(uint16_t)));
            HIP_TRY(c->PT.ensure((size_t)ldb * c->ldut * 2 * sizeof(uint16_t)));
        }
    }
    HIP_TRY(c->part.ensure((size_t)(fused && nrb > rp.nblk ? nrb : rp.nblk) * ldb * sizeof(double)));
    HIP_TRY(c->pre.ensure((size_t)2 * hd::kPreSplitRows * ldb * sizeof(double)));
    double *pre = c->pre.as<double>();
    HIP_TRY(c->scal.ensure((size_t)ldb * (5 * sizeof(double) + 3 * sizeof(int32_t)) + 128 * sizeof(int32_t)));
    HIP_TRY(c->err.ensure(sizeof(int32_t) * 4));
    {
        char *b = c->scal.as<char>();
        hd::CgState &st = c->st;
        st.rho0 = reinterpret_cast<double *>(b); b += ldb * sizeof(double);
        st.rho = reinterpret_cast<double *>(b); b += ldb * sizeof(double);
        st.a = reinterpret_cast<double *>(b); b += ldb * sizeof(double);
        st.beta = reinterpret_cast<double *>(b); b += ldb * sizeof(double);
        st.relres = reinterpret_cast<double *>(b); b += ldb * sizeof(double);
        st.active = reinterpret_cast<int32_t *>(b); b += ldb * sizeof(int32_t);
        st.iters = reinterpret_cast<int32_t *>(b); b += ldb * sizeof(int32_t);
        st.status = reinterpret_cast<int32_t *>(b); b += ldb * sizeof(int32_t);
        st.nact_part = reinterpret_cast<int32_t *>(b);
        st.maxit = nullptr;  // the host loop applies max_iter to every column
    }
    const hd::CgState st = c->st;

    // ---- step 1: observation vectors ----
    const int32_t *yi = y_ids;
    const float *yv = y_val;
    {
        const int e = queue_y(c, B, q_desc, y_ids, y_val, ky, y_ids_out, y_val_out, s, &yi, &yv);
        if (e != HD_OK) return e;
    }

    // ---- CG set-up: X = 0, R = P = y, rho0 = y^T y ----
    // With the dense bfloat16 forms and plain CG, the first iteration reads
    // R and P only on the rows of y (row mask) and X nowhere, and writes all
    // three everywhere: only the rows of y are zeroed before the scatter.
    // The other paths (fp32 or sparse U1, filters, no iteration) fill X, R
    // and P.
    float *X = c->X.as<float>(), *R = c->R.as<float>(), *P = c->P.as<float>(), *Q = c->Q.as<float>();
    const size_t nv = (size_t)n * ldb;
    const bool nofill = !flt && o->max_iter >= 1 && (fused || rk == 0);
    if (!nofill) {
        LAUNCH(K_FILL, hd::launch_fill_zero(X, nv, s));
        LAUNCH(K_FILL, hd::launch_fill_zero(R, nv, s));
        LAUNCH(K_FILL, hd::launch_fill_zero(P, nv, s));
    }
    LAUNCH(K_FILL, hd::launch_fill_zero(reinterpret_cast<float *>(c->err.p), 2, s));
    // the rows of y: the first product gathers only these rows of P (= y)
    const size_t nmask = (size_t)(n + 31) / 32;
    HIP_TRY(c->ymask.ensure(nmask * sizeof(uint32_t)));
    uint32_t *ymask = c->ymask.as<uint32_t>();
    LAUNCH(K_FILL, hd::launch_fill_zero(reinterpret_cast<float *>(ymask), nmask, s));
    if (nofill) LAUNCH(K_FILL, hd::launch_zero_yrows(B, ky, yi, n, ldb, R, P, s));
    LAUNCH(K_SCATTER, hd::launch_scatter_y(B, ky, yi, yv, n, ldb, R, P, c->err.as<int32_t>(), s, nullptr, ymask));
    LAUNCH(K_COLSQ, hd::launch_ynorm_part(B, ky, yi, n, ldb, R, c->part.as<double>(), s));
    LAUNCH(K_SCALAR, hd::launch_cg_init(B, ldb, c->part.as<double>(), 1, st, s));
    if (!graph) {
        HIP_TRY(hipMemcpyAsync(c->h_pinned + 200, c->err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(hipStreamSynchronize(s));
        if (c->timing.on) HIP_TRY(c->timing.harvest(0));
        if (c->h_pinned[200] != 0) return fail(HD_EINVAL, "hd_query_batch: a y id is outside [0, n)");
    }

    // ---- step 2: spectral coefficients (and L1 U1^T P for the first product) ----
    const bool ubf = c->u_mfma();
    const int64_t *Usr = c->Usr.as<int64_t>(), *Ustp = c->Ustp.as<int64_t>();
    const int32_t *Usc = c->Usc.as<int32_t>(), *Ustr = c->Ustr.as<int32_t>();
    const float *Usv = c->Usv.as<float>(), *Ustv = c->Ustv.as<float>();
    const float *U = c->U.as<float>();
    uint16_t *ClT_hi = c->ClT.as<uint16_t>(), *ClT_lo = ClT_hi ? ClT_hi + (size_t)rk * ldb : nullptr;
    uint16_t *CsT_hi = c->CsT.as<uint16_t>(), *CsT_lo = CsT_hi ? CsT_hi + (size_t)rk * ldb : nullptr;
    // a general filter's g(lambda_k) = h(lambda_k) - h(0) (Appendix A, eq. (2-aux))
    const double *gv = nullptr;
    if (flt && rk > 0) {
        std::vector<double> g((size_t)rk, 0.0);
        for (int k = 0; k < r_use; ++k) {
            double acc = 0.0, pw = 1.0;
            for (int i = 1; i <= flt->degree; ++i) {
                pw *= c->lam_host[(size_t)k];
                acc += flt->coeffs[i] * pw;
            }
            g[(size_t)k] = acc;
        }
        HIP_TRY(c->gfil.ensure(g.size() * sizeof(double)));
        HIP_TRY(hipMemcpy(c->gfil.p, g.data(), g.size() * sizeof(double), hipMemcpyHostToDevice));
        gv = c->gfil.as<double>();
    }
    if (rk > 0 && sparse) {
        LAUNCH(K_GATHER, hd::launch_sp_gather_proj(B, ky, yi, yv, n, Usr, Usc, Usv, rk, r_use, c->lam.as<double>(),
                                                   o->alpha, ldb, c->Cs.as<float>(), c->Cl.as<float>(), s,
                                                   nullptr, gv));
    } else if (rk > 0) {
        LAUNCH(K_GATHER, hd::launch_gather_proj(B, ky, yi, yv, n, ubf ? c->Ub.p : (const void *)U, c->ub_lo(),
                                                c->u_fmt(), c->rp, rk, r_use, c->lam.as<double>(), o->alpha,
                                                ldb, c->Cs.as<float>(), c->Cl.as<float>(), s, nullptr, gv,
                                                fused ? c->Dg.as<double>() : nullptr, c->u_scale()));
        if (ubf) {
            const hd::IterGuard none{nullptr, 0};
            LAUNCH(K_GATHER, hd::launch_split_t(c->Cs.as<float>(), rk, ldb, CsT_hi, CsT_lo, none, s));
            LAUNCH(K_GATHER, hd::launch_split_t(c->Cl.as<float>(), rk, ldb, ClT_hi, ClT_lo, none, s));
        }
    }

    // ---- step 3 (general filter, Appendix A, eq. (2-main)): the temporal
    // term h(S_r) y = sum_i c_i S_r^i y by Horner's rule, v = c_K y,
    // v = c_i y + S_r v. S_r v comes from the operator kernels with alpha = -1
    // and a zero P term: Z = -U1 L1 U1^T v, Q = (Z + S v) / 2 = S_r v / 2.
    const float *temporal = X;
    if (flt) {
        const hd::IterGuard none{nullptr, 0};
        const size_t nv2 = (size_t)n * ldb;
        float *Zb = rk > 0 ? c->Z.as<float>() : nullptr;
        LAUNCH(K_UPDATE_XP, hd::launch_filter_axpy(P, R, Q, nv2, flt->coeffs[flt->degree], 0.0, s));
        for (int i = flt->degree - 1; i >= 0; --i) {
            const float *Zs = X;  // zeros
            if (rk > 0) {
                if (sparse) {
                    LAUNCH(K_UT_P, hd::launch_sp_utp(rk, r_use, Ustp, Ustr, Ustv, P, ldb, c->lam.as<double>(),
                                                     c->Cl.as<float>(), none, s));
                    LAUNCH(K_U_C, hd::launch_sp_uc(n, Usr, Usc, Usv, c->Cl.as<float>(), ldb, X, -1.0, Zb, none, s));
                } else {
                    if (ubf) {
                        uint16_t *PTh = c->PT.as<uint16_t>(), *PTl = PTh + (size_t)ldb * c->ldut;
                        LAUNCH(K_UT_P, hd::launch_split_pt(n, ldb, P, c->ldut, PTh, PTl, none, s));
                        LAUNCH(K_UT_P, hd::launch_ut_p_bf16(n, c->u_comp(), c->ldut, rk, PTh, PTl, ldb,
                                                            c->Cpart.as<float>(), none, s, c->tv(HD_TUNE_UTP_NT, ldb)));
                    } else {
                        LAUNCH(K_UT_P, hd::launch_ut_p(n, U, c->rp, rk, P, ldb, c->Cpart.as<float>(), none, s));
                    }
                    LAUNCH(K_REDUCE_C, hd::launch_reduce_c(nchunk, c->Cpart.as<float>(), rk, ldb, c->lam.as<double>(),
                                                           r_use, c->Cl.as<float>(), none, s, nullptr, 0.0,
                                                           c->u_scale()));
                    if (ubf) {
                        LAUNCH(K_REDUCE_C, hd::launch_split_t(c->Cl.as<float>(), rk, ldb, ClT_hi, ClT_lo, none, s));
                        LAUNCH(K_U_C, hd::launch_u_c_bf16(n, c->u_item(), c->rp, rk, ClT_hi, ClT_lo, ldb, X, -1.0, Zb,
                                                          none, s, c->tv(HD_TUNE_UC_NT, ldb)));
                    } else {
                        LAUNCH(K_U_C, hd::launch_u_c(n, U, c->rp, rk, c->Cl.as<float>(), ldb, X, -1.0, Zb, none, s));
                    }
                }
                Zs = Zb;
            }
            LAUNCH(K_SPMM, hd::launch_spmm(n, c->rowptr.as<int64_t>(), c->col.as<int32_t>(), c->val.as<float>(), P, Zs,
                                           Q, ldb, -1.0, rp, c->part.as<double>(), none, s,
                                           c->tv(HD_TUNE_SPMM_CPL, ldb), 0, nullptr, c->bands(), c->cuts()));
            LAUNCH(K_UPDATE_XP, hd::launch_filter_axpy(P, R, Q, nv2, flt->coeffs[i], 2.0, s));
        }
        temporal = P;
    }

    // ---- step 3: CG on the deflated system ----
    // Iteration it checks the active counts left by iteration it-1 (parity
    // (it-1)&1) and its stopping test writes parity it&1, which is copied to
    // pinned memory behind an event. The host queues iteration it+1 before
    // waiting for iteration it's counts, so the GPU never idles on the host;
    // an iteration queued after the last one returns at once from every kernel.
    // In graph form all max_iter iterations are queued with no host
    // synchronisation: the same guards turn the iterations after the last
    // active one into empty kernels.
    const int ntile = ldb / 64;
    int32_t *nact_dev[2] = {st.nact_part, st.nact_part + 64};
    // the last iteration's x update (x += a p; nothing reads the new P) is
    // left to the combine when its kernel can apply it (the two-term, bf16
    // and fp8 U1 forms, and r = 0) and x is read at all; it is not for one
    // iteration, whose update runs with the row mask of y
    const bool xfold = !flt && o->max_iter >= 2 &&
                       (rk == 0 || (ubf && !sparse && hd::combine_nt(ldb, c->tv(HD_TUNE_UC_NT, ldb)) != 4)) &&
                       (x_out || (o->top_k > 0 && (rank_ids || rank_scores)));
    auto enqueue_iter = [&](int it) -> int {
        c->timing.tag = it;
        const hd::IterGuard g{nact_dev[(it - 1) & 1], ntile};
        // first iteration without fills: the updates read R and P on the
        // rows of y only, and always run (they write X, R and P everywhere;
        // a = 0 leaves a stopped column's values as they are)
        const bool m1 = nofill && it == 1;
        const uint32_t *rm = m1 ? ymask : nullptr;
        const hd::IterGuard gu = m1 ? hd::IterGuard{nullptr, 0} : g;
        // tol < 0: the last product forms no residual (x alone is updated)
        const bool nores = o->tol < 0.0 && it == o->max_iter;
        if (fused) {
            uint16_t *PTh = c->PT.as<uint16_t>(), *PTl = PTh + (size_t)ldb * c->ldut;
            if (it > 1) {
                // L1 U1^T P (P^T split written by the previous iteration's
                // update) and the eigenvector part of gamma
                LAUNCH(K_UT_P, hd::launch_ut_p_bf16(n, c->u_comp(), c->ldut, rk, PTh, PTl, ldb, c->Cpart.as<float>(),
                                                    g, s, c->tv(HD_TUNE_UTP_NT, ldb)));
                LAUNCH(K_REDUCE_C, hd::launch_reduce_c(nchunk, c->Cpart.as<float>(), rk, ldb, c->lam.as<double>(),
                                                       r_use, c->Cl.as<float>(), g, s, c->Dg.as<double>(),
                                                       o->alpha, c->u_scale()));
                LAUNCH(K_REDUCE_C, hd::launch_split_t(c->Cl.as<float>(), rk, ldb, ClT_hi, ClT_lo, g, s));
            }
            LAUNCH(it == 1 ? K_SPMM_Y : K_SPMM,
                   hd::launch_spmm(n, c->rowptr.as<int64_t>(), c->col.as<int32_t>(), c->val.as<float>(), P, P, Q,
                                   ldb, o->alpha, rp, c->part.as<double>(), g, s, c->tv(HD_TUNE_SPMM_CPL, ldb), 0,
                                   it == 1 ? ymask : nullptr, c->bands(), c->cuts()));
            LAUNCH(K_SCALAR, hd::launch_cg_step_a(ldb, c->part.as<double>(), rp.nblk, st, g, s, c->Dg.as<double>(),
                                                  rk, pre));
            if (!nores)
                LAUNCH(K_U_C, hd::launch_uc_update_r_bf16(n, c->u_item(), c->rp, rk, ClT_hi, ClT_lo, ldb, Q, o->alpha,
                                                          R, st.a, c->part.as<double>(), gu, s,
                                                          c->tv(HD_TUNE_UC_NT, ldb), 0, rm));
            LAUNCH(K_SCALAR, hd::launch_cg_step_b(ldb, nores ? nullptr : c->part.as<double>(), nrb, o->tol, st, g,
                                                  nact_dev[it & 1], s, pre));
            if (it == o->max_iter) {  // nothing reads the new P or its split transpose
                if (!xfold)
                    LAUNCH(K_UPDATE_XP, hd::launch_update_xp(n, ldb, X, P, R, st.a, st.beta, st.active, gu, s, 0,
                                                             true, rm));
            } else
                LAUNCH(K_UPDATE_XP, hd::launch_update_xp_pt(n, ldb, X, P, R, st.a, st.beta, st.active, c->ldut,
                                                            PTh, PTl, gu, s, rm));
            if (!graph) {
                HIP_TRY(hipMemcpyAsync(c->h_pinned + 64 * (it & 1), nact_dev[it & 1], ntile * sizeof(int32_t),
                                       hipMemcpyDeviceToHost, s));
                HIP_TRY(hipEventRecord(c->iter_ev[it & 1], s));
            }
            c->timing.tag = 0;
            return HD_OK;
        }
        const float *Zs = P;
        if (rk > 0 && sparse) {
            if (it > 1)
                LAUNCH(K_UT_P, hd::launch_sp_utp(rk, r_use, Ustp, Ustr, Ustv, P, ldb, c->lam.as<double>(),
                                                 c->Cl.as<float>(), g, s));
            LAUNCH(K_U_C, hd::launch_sp_uc(n, Usr, Usc, Usv, c->Cl.as<float>(), ldb, P, o->alpha, c->Z.as<float>(),
                                           g, s));
            Zs = c->Z.as<float>();
        } else if (rk > 0) {
            if (it > 1) {
                if (ubf) {
                    // PT was written by the previous iteration's update_xp
                    uint16_t *PTh = c->PT.as<uint16_t>(), *PTl = PTh + (size_t)ldb * c->ldut;
                    LAUNCH(K_UT_P, hd::launch_ut_p_bf16(n, c->u_comp(), c->ldut, rk, PTh, PTl, ldb,
                                                        c->Cpart.as<float>(), g, s, c->tv(HD_TUNE_UTP_NT, ldb)));
                } else {
                    LAUNCH(K_UT_P, hd::launch_ut_p(n, U, c->rp, rk, P, ldb, c->Cpart.as<float>(), g, s));
                }
                LAUNCH(K_REDUCE_C, hd::launch_reduce_c(nchunk, c->Cpart.as<float>(), rk, ldb, c->lam.as<double>(),
                                                       r_use, c->Cl.as<float>(), g, s, nullptr, 0.0, c->u_scale()));
                if (ubf) LAUNCH(K_REDUCE_C, hd::launch_split_t(c->Cl.as<float>(), rk, ldb, ClT_hi, ClT_lo, g, s));
            }
            if (ubf) {
                LAUNCH(K_U_C, hd::launch_u_c_bf16(n, c->u_item(), c->rp, rk, ClT_hi, ClT_lo, ldb, P, o->alpha,
                                                  c->Z.as<float>(), g, s, c->tv(HD_TUNE_UC_NT, ldb)));
            } else {
                LAUNCH(K_U_C, hd::launch_u_c(n, U, c->rp, rk, c->Cl.as<float>(), ldb, P, o->alpha, c->Z.as<float>(), g, s));
            }
            Zs = c->Z.as<float>();
        }
        LAUNCH(it == 1 ? K_SPMM_Y : K_SPMM,
               hd::launch_spmm(n, c->rowptr.as<int64_t>(), c->col.as<int32_t>(), c->val.as<float>(), P, Zs, Q, ldb,
                               o->alpha, rp, c->part.as<double>(), g, s, c->tv(HD_TUNE_SPMM_CPL, ldb), 0,
                               it == 1 ? ymask : nullptr, c->bands(), c->cuts()));
        LAUNCH(K_SCALAR, hd::launch_cg_step_a(ldb, c->part.as<double>(), rp.nblk, st, g, s, nullptr, 0, pre));
        if (!nores) LAUNCH(K_UPDATE_R, hd::launch_update_r(n, ldb, Q, R, rp, st.a, c->part.as<double>(), gu, s, rm));
        LAUNCH(K_SCALAR, hd::launch_cg_step_b(ldb, nores ? nullptr : c->part.as<double>(), rp.nblk, o->tol, st, g,
                                              nact_dev[it & 1], s, pre));
        if (it == o->max_iter) {  // the last iteration: nothing reads the new P
            if (!xfold)
                LAUNCH(K_UPDATE_XP, hd::launch_update_xp(n, ldb, X, P, R, st.a, st.beta, st.active, gu, s, 0, true,
                                                         rm));
        } else if (ubf && rk > 0) {
            uint16_t *PTh = c->PT.as<uint16_t>(), *PTl = PTh + (size_t)ldb * c->ldut;
            LAUNCH(K_UPDATE_XP, hd::launch_update_xp_pt(n, ldb, X, P, R, st.a, st.beta, st.active, c->ldut,
                                                        PTh, PTl, gu, s, rm));
        } else {
            LAUNCH(K_UPDATE_XP, hd::launch_update_xp(n, ldb, X, P, R, st.a, st.beta, st.active, gu, s, 0, false, rm));
        }
        if (!graph) {
            HIP_TRY(hipMemcpyAsync(c->h_pinned + 64 * (it & 1), nact_dev[it & 1], ntile * sizeof(int32_t),
                                   hipMemcpyDeviceToHost, s));
            HIP_TRY(hipEventRecord(c->iter_ev[it & 1], s));
        }
        c->timing.tag = 0;
        return HD_OK;
    };
    int last_iter = 0;
    if (flt) {
        // no CG: the temporal term is already in P
    } else if (graph) {
        for (int it = 1; it <= o->max_iter; ++it) {
            const int e = enqueue_iter(it);
            if (e != HD_OK) return e;
        }
        last_iter = o->max_iter;
    } else if (o->max_iter >= 1) {
        const int e = enqueue_iter(1);
        if (e != HD_OK) return e;
    }
    for (int it = 1; !flt && !graph && it <= o->max_iter; ++it) {
        if (it + 1 <= o->max_iter) {
            const int e = enqueue_iter(it + 1);
            if (e != HD_OK) return e;
        }
        HIP_TRY(hipEventSynchronize(c->iter_ev[it & 1]));
        last_iter = it;
        int nact = 0;
        for (int t = 0; t < ntile; ++t) nact += c->h_pinned[64 * (it & 1) + t];
        if (nact == 0) break;
    }
    LAUNCH(K_SCALAR, hd::launch_cg_final(ldb, st, s));

    // ---- step 4: x = x^s + x^t (query-major), ranking ----
    float *xq = x_out;
    if (!xq) {
        HIP_TRY(c->xbuf.ensure((size_t)B * n * sizeof(float)));
        xq = c->xbuf.as<float>();
    }
    const bool rank = o->top_k > 0 && (rank_ids || rank_scores);
    const int K = o->top_k;
    // the last iteration's x update, when it was left to the combine
    const hd::XFold xf{st.a, P, hd::IterGuard{nact_dev[(o->max_iter - 1) & 1], ntile}};
    const hd::XFold *fold = xfold ? &xf : nullptr;
    if (rank && !x_out && (rk == 0 || (ubf && !sparse)) && c->onepass_rank(rk)) {
        // one-pass ranking: thresholds from the sampled items' x, then the
        // combine offers every x to the lists without writing x; xq is
        // written only if some row needs the exact fallback
        int64_t st, m;
        hd::topk_sample(n, &st, &m);
        const int64_t lss = (m + 63) / 64 * 64;
        HIP_TRY(c->topk.ensure(hd::topk_scratch_bytes(B, n, K)));
        HIP_TRY(c->tsx.ensure(onepass_sample_bytes(B, m)));
        float *ss = c->tsx.as<float>(), *xs = ss + (size_t)B * lss;
        const hd::TopkLists tl = hd::topk_lists(c->topk.p, B, n);
        const int32_t *gate = hd::topk_fallback_gate(c->topk.p, B, n);
        const int nt = c->tv(HD_TUNE_UC_NT, ldb);
        LAUNCH(K_TOPK_RANK, hd::launch_sample_rows(m, st, ldb, temporal, xs, s, fold));
        if (rk > 0) {
            LAUNCH(K_TOPK_RANK, hd::launch_combine_bf16(m, B, c->u_item_sample(), c->rp, rk, CsT_hi, CsT_lo, ldb, xs,
                                                          ss, lss, s, nt));
            LAUNCH(K_TOPK_RANK, hd::launch_topk_prepare(B, n, ss, lss, 1, K, c->topk.p, s));
            LAUNCH(K_COMBINE, hd::launch_combine_bf16(n, B, c->u_item(), c->rp, rk, CsT_hi, CsT_lo, ldb, temporal,
                                                        nullptr, n, s, nt, &tl, nullptr, fold));
        } else {
            LAUNCH(K_TOPK_RANK, hd::launch_topk_prepare(B, n, xs, 1, ldb, K, c->topk.p, s));
            LAUNCH(K_COMBINE, hd::launch_topk_emit_nm(n, B, ldb, temporal, tl, s, fold));
        }
        LAUNCH(K_TOPK_RANK, hd::launch_topk_select_lists(B, n, K, c->topk.p, rank_ids, rank_scores, 0, s));
        if (rk > 0) {
            LAUNCH(K_TOPK_RANK, hd::launch_combine_bf16(n, B, c->u_item(), c->rp, rk, CsT_hi, CsT_lo, ldb, temporal, xq,
                                                          n, s, nt, nullptr, gate, fold));
        } else {
            LAUNCH(K_TOPK_RANK, hd::launch_combine(n, B, nullptr, c->rp, 0, nullptr, ldb, temporal, xq, n, s, gate,
                                                   fold));
        }
        LAUNCH(K_TOPK_RANK, hd::launch_topk_fallback(B, n, xq, n, K, c->topk.p, rank_ids, rank_scores, 0, s));
    } else {
        if (x_out || o->top_k > 0) {
            if (sparse && rk > 0) {
                LAUNCH(K_COMBINE, hd::launch_sp_combine(n, B, Usr, Usc, Usv, c->Cs.as<float>(), ldb, temporal, xq, n, s));
            } else if (ubf && rk > 0) {
                LAUNCH(K_COMBINE, hd::launch_combine_bf16(n, B, c->u_item(), c->rp, rk, CsT_hi, CsT_lo, ldb, temporal,
                                                            xq, n, s, c->tv(HD_TUNE_UC_NT, ldb), nullptr, nullptr,
                                                            fold));
            } else {
                LAUNCH(K_COMBINE, hd::launch_combine(n, B, U, c->rp, rk, c->Cs.as<float>(), ldb, temporal, xq, n, s,
                                                     nullptr, rk == 0 ? fold : nullptr));
            }
        }
        if (rank) {
            HIP_TRY(c->topk.ensure(hd::topk_scratch_bytes(B, n, K)));
            LAUNCH(K_TOPK_RANK, hd::launch_topk(B, n, xq, n, K, c->topk.p, rank_ids, rank_scores, 0, s));
        }
    }
    if (last_iter_out) *last_iter_out = last_iter;
    return HD_OK;
}

extern "C" {

int hd_query_filter(hd_ctx *c, int32_t B, const float *q_desc, const int32_t *y_ids, const float *y_val,
                    int32_t degree, const double *coeffs, int32_t rank_r, int32_t k_y, int32_t top_k,
                    int32_t *rank_ids, float *rank_scores, float *x_out, void *stream) {
    g_err.clear();
    if (degree < 0 || degree > 4096) return fail(HD_EINVAL, "hd_query_filter: degree=%d not in [0, 4096]", degree);
    if (!coeffs) return fail(HD_EINVAL, "hd_query_filter: NULL coefficients");
    for (int i = 0; i <= degree; ++i)
        if (!std::isfinite(coeffs[i])) return fail(HD_EINVAL, "hd_query_filter: coefficient %d not finite", i);
    hd_query_opts o{0.5, 0, 0.0, rank_r, k_y, top_k};
    const Filter f{degree, coeffs};
    hipStream_t s = (hipStream_t)stream;
    const int e = queue_query(c, B, q_desc, y_ids, y_val, &o, rank_ids, rank_scores, x_out, nullptr, nullptr, s,
                              false, nullptr, &f);
    if (e != HD_OK) return e;
    HIP_TRY(hipStreamSynchronize(s));
    if (c->timing.on) HIP_TRY(c->timing.harvest(0));
    return HD_OK;
}

int hd_query_batch(hd_ctx *c, int32_t B, const float *q_desc, const int32_t *y_ids,
                   const float *y_val, const hd_query_opts *o, int32_t *rank_ids,
                   float *rank_scores, float *x_out, int32_t *y_ids_out, float *y_val_out,
                   int32_t *iters, double *relres, int32_t *status, void *stream) {
    g_err.clear();
    hipStream_t s = (hipStream_t)stream;
    int last_iter = 0;
    const int e = queue_query(c, B, q_desc, y_ids, y_val, o, rank_ids, rank_scores, x_out, y_ids_out,
                              y_val_out, s, false, &last_iter);
    if (e != HD_OK) return e;
    const hd::CgState &st = c->st;
    if (iters) HIP_TRY(hipMemcpyAsync(iters, st.iters, B * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (status) HIP_TRY(hipMemcpyAsync(status, st.status, B * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (relres) HIP_TRY(hipMemcpyAsync(relres, st.relres, B * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (c->timing.on) HIP_TRY(c->timing.harvest(last_iter));
    return HD_OK;
}

}  // extern "C"
