// Launch parameters of the hot kernels and the autotuner that picks them.
//
// The search space is small and discrete (columns per lane of the sparse
// product; 16-column tiles per wave of the bfloat16 eigenvector products),
// so the tuner times every candidate on the context's own graph and
// eigenvectors at the solver width of the batch size it is asked for, on
// scratch vectors, and keeps the fastest. Timing uses HIP events on the
// null stream around `reps` back-to-back launches after one warm-up launch.
// A candidate replaces the built-in default only when it is more than 2%
// faster: near-equal candidates would otherwise flip between runs on timing
// noise, and the chosen launch variant decides which kernel a profile counts.
#include "hd_internal.h"

namespace {

// the value each launcher picks for tuning value 0 at solver width ldb
int default_value(int key, int ldb) {
    const int cap = key == HD_TUNE_SPMM_CPL ? 2 : key == HD_TUNE_UTP_NT ? 4 : 2;
    for (int v = cap; v > 1; v /= 2)
        if (ldb % (64 * v) == 0) return v;
    return 1;
}

constexpr double kKeepDefault = 0.98;
// more than one source band of the sparse product: only when 5% faster than
// one pass (on graphs without locality the bands add work and no cache hits;
// a 2% margin let timing noise pick them)
constexpr double kKeepBands = 0.95;

}  // namespace

extern "C" {

int hd_set_tuning(hd_ctx *c, int32_t key, int32_t value) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_set_tuning: NULL context");
    if (key < 0 || key >= HD_TUNE_NKEYS) return fail(HD_EINVAL, "hd_set_tuning: key %d unknown", key);
    if (key == HD_TUNE_SPMM_BANDS) {
        if (value != 0 && !hd::band_param_ok(value))
            return fail(HD_EINVAL, "hd_set_tuning: value %d not in {0, 1, 2, 4, 8}", value);
    } else if (key == HD_TUNE_TOPK_ONEPASS) {
        if (value < 0 || value > 2) return fail(HD_EINVAL, "hd_set_tuning: value %d not in {0, 1, 2}", value);
    } else if (value != 0 && value != 1 && value != 2 && value != 4) {
        return fail(HD_EINVAL, "hd_set_tuning: value %d not in {0, 1, 2, 4}", value);
    }
    c->tune[key] = value;
    return HD_OK;
}

int hd_get_tuning(const hd_ctx *c, int32_t key, int32_t *value) {
    g_err.clear();
    if (!c || !value) return fail(HD_EINVAL, "hd_get_tuning: NULL argument");
    if (key < 0 || key >= HD_TUNE_NKEYS) return fail(HD_EINVAL, "hd_get_tuning: key %d unknown", key);
    *value = c->tune[key];
    return HD_OK;
}

int hd_autotune(hd_ctx *c, int32_t batch, int32_t reps, double *times_ms) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_autotune: NULL context");
    if (c->n == 0) return fail(HD_ESTATE, "hd_autotune: no graph loaded");
    if (batch < 1 || batch > 1024) return fail(HD_EINVAL, "hd_autotune: batch=%d not in [1, 1024]", batch);
    if (reps < 1 || reps > 1000) return fail(HD_EINVAL, "hd_autotune: reps=%d not in [1, 1000]", reps);
    HIP_TRY(hipSetDevice(c->device));
    const int64_t n = c->n;
    const int ldb = pow2_at_least(batch);
    const int rk = c->rp;
    const bool ubf = c->u_mfma() && rk > 0;
    const size_t vec = (size_t)n * ldb * sizeof(float);
    const hd::RowPart rp = hd::make_row_part(n);
    int64_t rc;
    const int nchunk = hd::ut_p_chunks(n, &rc);
    HIP_TRY(c->P.ensure(vec));
    HIP_TRY(c->Q.ensure(vec));
    HIP_TRY(c->Z.ensure(vec));
    const int nrb = hd::uc_update_r_blocks(n);
    HIP_TRY(c->part.ensure((size_t)(nrb > rp.nblk ? nrb : rp.nblk) * ldb * sizeof(double)));
    hipStream_t s = nullptr;
    HIP_TRY(hd::launch_fill_zero(c->P.as<float>(), (size_t)n * ldb, s));
    HIP_TRY(hd::launch_fill_zero(c->Q.as<float>(), (size_t)n * ldb, s));
    HIP_TRY(hd::launch_fill_zero(c->Z.as<float>(), (size_t)n * ldb, s));
    uint16_t *PTh = nullptr, *PTl = nullptr, *CTh = nullptr, *CTl = nullptr;
    if (ubf) {
        HIP_TRY(c->Cpart.ensure((size_t)nchunk * rk * ldb * sizeof(float)));
        HIP_TRY(c->ClT.ensure((size_t)rk * ldb * 2 * sizeof(uint16_t)));
        HIP_TRY(c->PT.ensure((size_t)ldb * c->ldut * 2 * sizeof(uint16_t)));
        PTh = c->PT.as<uint16_t>();
        PTl = PTh + (size_t)ldb * c->ldut;
        CTh = c->ClT.as<uint16_t>();
        CTl = CTh + (size_t)rk * ldb;
        HIP_TRY(hd::launch_fill_zero(reinterpret_cast<float *>(CTh), (size_t)rk * ldb, s));
        // per-column CG step sizes of the timed residual updates (zero)
        HIP_TRY(c->Dg.ensure((size_t)rk * ldb * sizeof(double)));
        HIP_TRY(hd::launch_fill_zero(c->Dg.as<float>(), (size_t)rk * ldb * 2, s));
        HIP_TRY(hd::launch_split_pt(n, ldb, c->P.as<float>(), c->ldut, PTh, PTl, hd::IterGuard{nullptr, 0}, s));
    }
    const hd::IterGuard none{nullptr, 0};
    // v: the key's value; bands: the sparse product's source bands
    auto launch = [&](int key, int v, int bands) -> hipError_t {
        switch (key) {
        case HD_TUNE_SPMM_CPL:
            return hd::launch_spmm(n, c->rowptr.as<int64_t>(), c->col.as<int32_t>(), c->val.as<float>(),
                                   c->P.as<float>(), c->Z.as<float>(), c->Q.as<float>(), ldb, 0.99, rp,
                                   c->part.as<double>(), none, s, v, 0, nullptr, bands, c->cuts());
        case HD_TUNE_UTP_NT:
            return hd::launch_ut_p_bf16(n, c->u_comp(), c->ldut, rk, PTh, PTl, ldb,
                                        c->Cpart.as<float>(), none, s, v);
        default:
            // U C as it runs in CG: fused with the residual update
            return hd::launch_uc_update_r_bf16(n, c->u_item(), c->rp, rk, CTh, CTl, ldb,
                                               c->Q.as<float>(), 0.99, c->Z.as<float>(), c->Dg.as<double>(),
                                               c->part.as<double>(), none, s, v);
        }
    };
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    const int cand[4] = {1, 2, 4, 8};
    int err = HD_OK;
    // mean ms of one launch (one warm-up first); < 0 on error
    auto time_one = [&](int key, int v, int bands) -> double {
        hipError_t e = launch(key, v, bands);
        if (e == hipSuccess) e = hipEventRecord(e0, s);
        for (int t = 0; t < reps && e == hipSuccess; ++t) e = launch(key, v, bands);
        if (e == hipSuccess) e = hipEventRecord(e1, s);
        if (e == hipSuccess) e = hipEventSynchronize(e1);
        float el = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&el, e0, e1);
        if (e != hipSuccess) {
            err = fail(HD_EDEVICE, "hd_autotune: %s", hipGetErrorString(e));
            return -1.0;
        }
        return (double)el / reps;
    };
    if (times_ms)
        for (int j = 0; j < 4 * HD_TUNE_NKEYS; ++j) times_ms[j] = -1.0;
    // the sparse product: every (columns per lane, bands) pair
    {
        double t[3][4];
        double best = -1.0;
        int bc = 0, bb = 0;
        const int def_c = default_value(HD_TUNE_SPMM_CPL, ldb), def_b = 1;
        double def_ms = -1.0;
        for (int i = 0; i < 3 && err == HD_OK; ++i)
            for (int j = 0; j < 4 && err == HD_OK; ++j) {
                t[i][j] = -1.0;
                if (!hd::tile_param_ok(cand[i], ldb)) continue;
                const double ms = time_one(HD_TUNE_SPMM_CPL, cand[i], cand[j]);
                if (ms < 0.0) break;
                t[i][j] = ms;
                if (cand[i] == def_c && cand[j] == def_b) def_ms = ms;
                if (best < 0.0 || ms < best) {
                    best = ms;
                    bc = i;
                    bb = j;
                }
            }
        if (err == HD_OK && best >= 0.0) {
            // one pass first: the fastest column tiling unless the default is
            // within 2%; more bands only when they beat that by more than 5%
            double b1 = -1.0;
            int c1 = 0;
            for (int i = 0; i < 3; ++i)
                if (t[i][0] >= 0.0 && (b1 < 0.0 || t[i][0] < b1)) {
                    b1 = t[i][0];
                    c1 = i;
                }
            if (def_ms >= 0.0 && b1 >= kKeepDefault * def_ms) {
                b1 = def_ms;
                c1 = def_c == 1 ? 0 : def_c == 2 ? 1 : 2;
            }
            const bool banded = bb > 0 && b1 >= 0.0 && best < kKeepBands * b1;
            const int ci = banded ? bc : c1, bi = banded ? bb : 0;
            c->tune[HD_TUNE_SPMM_CPL] = cand[ci];
            c->tune[HD_TUNE_SPMM_BANDS] = cand[bi];
            if (times_ms) {
                for (int i = 0; i < 3; ++i) times_ms[HD_TUNE_SPMM_CPL * 4 + i] = t[i][bi];
                for (int j = 0; j < 4; ++j) times_ms[HD_TUNE_SPMM_BANDS * 4 + j] = t[ci][j];
            }
        }
    }
    for (int key : {HD_TUNE_UTP_NT, HD_TUNE_UC_NT}) {
        if (err != HD_OK || !ubf) break;
        double best = -1.0, def_ms = -1.0;
        int best_v = 0;
        const int def_v = default_value(key, ldb);
        for (int j = 0; j < 3; ++j) {
            if (!hd::tile_param_ok(cand[j], ldb)) continue;
            const double ms = time_one(key, cand[j], 1);
            if (ms < 0.0) break;
            if (cand[j] == def_v) def_ms = ms;
            if (best < 0.0 || ms < best) {
                best = ms;
                best_v = cand[j];
            }
            if (times_ms) times_ms[key * 4 + j] = ms;
        }
        if (err == HD_OK && best_v != 0)
            c->tune[key] = (def_ms >= 0.0 && best >= kKeepDefault * def_ms) ? def_v : best_v;
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return err;
}

}  // extern "C"
