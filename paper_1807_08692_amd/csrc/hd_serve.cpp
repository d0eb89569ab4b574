// Continuous-batching server (C ABI hd_serve_*, declared in include/hd.h).
//
// A server keeps one conjugate-gradient solve running over `slots` query
// columns of the context's graph and eigenpairs. Requests are admitted into
// free columns between iterations - while other columns are in the middle of
// their own solves - and leave when their column stops (converged, its own
// iteration cap, zero right-hand side or breakdown): the combine and top-K
// ranking then run for the finished columns only and the columns are freed.
// Every column is an independent CG recurrence with fixed-order reductions,
// so a request's result does not depend on which other requests share the
// solve. The number of columns is chosen against an HBM budget at open time.
#include "hd_internal.h"

#include <vector>

namespace {

struct Srv {
    hd_ctx *c = nullptr;
    hd_query_opts o{};
    std::vector<intptr_t> data;  // the context's data the server was opened on
    int slots = 0, ldb = 0, rk = 0, r_use = 0;
    hipStream_t s = nullptr;
    // bfloat16 U1: the eigenvector correction follows the sparse product and
    // goes into the residual update, as in the batch path
    bool fused = false;
    hd::RowPart rp{};
    int nchunk = 0, nrb = 0;
    DevBuf X, R, P, Q, Z, Cpart, Cl, Cs, ClT, CsT, PT, part, scal, err, cols, maxit, xc, csc, cst, xq,
        topk, rids, rsc, ybuf, qbuf, sim, qsplit, Dg;
    hd::CgState st{};
    int32_t *h = nullptr;  // pinned: [0,ldb) active, [ldb,2ldb) iters, [2ldb,3ldb) status, err
    double *hr = nullptr;  // pinned: relres
    std::vector<int64_t> ticket;  // per column, -1 = free
    // per column (bfloat16 forms): 1 = its X, R, P may hold values that no
    // step has cleared since a request was admitted into it or stopped
    // outside a step (cancelled); admission clears such a column first. A
    // column whose request stops inside a step is cleared by that step's
    // x/p update (launch_update_xp_pt with the iteration counts).
    std::vector<uint8_t> dirty;
    int64_t next_ticket = 1;

    void release() {
        DevBuf *all[] = {&X, &R, &P, &Q, &Z, &Cpart, &Cl, &Cs, &ClT, &CsT, &PT, &part, &scal, &err, &cols,
                         &maxit, &xc, &csc, &cst, &xq, &topk, &rids, &rsc, &ybuf, &qbuf, &sim,
                         &qsplit, &Dg};
        for (DevBuf *b : all) b->release();
        if (h) (void)hipHostFree(h);
        if (hr) (void)hipHostFree(hr);
        if (s) (void)hipStreamDestroy(s);
        h = nullptr;
        hr = nullptr;
        s = nullptr;
    }
};

// Device bytes one solver column needs at n items (vectors X R P Q, and Z
// for fp32 U1, the coefficient columns, the partial sums and the ranking
// buffers).
int64_t bytes_per_column(const hd_ctx *c, int rk, int nchunk, int nblk, int top_k, int ky) {
    // the vectors, the partial and full coefficient columns, reduction
    // partials (and the eigenvector part of gamma), the gathered x columns,
    // the split P^T of the bfloat16 forms
    const bool fused = c->u_mfma() && rk > 0;
    const int64_t nrb = hd::uc_update_r_blocks(c->n);
    const int64_t prow = fused && nrb > nblk ? nrb : nblk;
    const int64_t kmax = ky > top_k ? ky : top_k;
    // the top-k scratch of one row (y selection or ranking), and, when the
    // requests come as descriptors, the row of similarities, the query and
    // its bfloat16 split
    const int64_t topk_row = (int64_t)hd::topk_scratch_bytes(1, c->n, (int)kmax);
    const int64_t desc = c->d > 0 ? 4 * ((c->n + 63) / 64 * 64) + 4 * (int64_t)c->d + 4 * (int64_t)c->ldv : 0;
    return (fused ? 4 : 5) * 4 * c->n + (int64_t)4 * rk * (nchunk + 4) + 8 * prow + (fused ? 8 * rk : 0) +
           4 * c->n * 2 + (fused ? 4 * c->ldut : 0) + (int64_t)top_k * 8 + (int64_t)ky * 8 + topk_row + desc +
           64;
}

// The context's loaded data and layouts; a server refuses to run once they
// have changed (its buffers are sized for what it was opened on).
std::vector<intptr_t> data_of(const hd_ctx *c) {
    return {(intptr_t)c->n, (intptr_t)c->nnz, (intptr_t)c->r, (intptr_t)c->rp, (intptr_t)c->u_dtype,
            (intptr_t)c->ldut, (intptr_t)c->d, (intptr_t)c->ldv, (intptr_t)c->v_dtype,
            (intptr_t)c->rowptr.p, (intptr_t)c->U.p, (intptr_t)c->Ub.p, (intptr_t)c->UbT.p,
            (intptr_t)c->lam.p, (intptr_t)c->V.p, (intptr_t)c->Vb.p, (intptr_t)c->uscale.p,
            (intptr_t)c->vscale.p};
}

}  // namespace

struct hd_server : Srv {};

extern "C" {

int hd_serve_open(hd_ctx *c, int32_t slots, int64_t hbm_budget_bytes, const hd_query_opts *o,
                  hd_server **out) {
    g_err.clear();
    if (!out) return fail(HD_EINVAL, "hd_serve_open: out is NULL");
    *out = nullptr;
    if (!c || !o) return fail(HD_EINVAL, "hd_serve_open: NULL context or options");
    if (c->n == 0) return fail(HD_ESTATE, "hd_serve_open: no graph loaded");
    if (slots < 1 || slots > 1024) return fail(HD_EINVAL, "hd_serve_open: slots=%d not in [1, 1024]", slots);
    if (!(o->alpha >= 0.0 && o->alpha < 1.0)) return fail(HD_EINVAL, "hd_serve_open: alpha=%g not in [0, 1)", o->alpha);
    if (o->max_iter < 0 || std::isnan(o->tol)) return fail(HD_EINVAL, "hd_serve_open: bad max_iter or tol");
    if (o->k_y < 1 || o->k_y > c->n || o->k_y > hd::kTopkMax) return fail(HD_EINVAL, "hd_serve_open: bad k_y");
    if (o->top_k < 1 || o->top_k > c->n || o->top_k > hd::kTopkMax)
        return fail(HD_EINVAL, "hd_serve_open: top_k must be in [1, min(n, 1024)]");
    const int r_use = o->rank_r < 0 ? c->r : o->rank_r;
    if (r_use > c->r) return fail(HD_ESTATE, "hd_serve_open: rank_r=%d above the %d loaded eigenpairs", r_use, c->r);
    if (r_use > 0 && c->u_sparse())
        return fail(HD_ESTATE, "hd_serve_open: the server does not take sparsified eigenvectors");
    HIP_TRY(hipSetDevice(c->device));
    const int rk = (r_use + 31) / 32 * 32;
    const hd::RowPart rp = hd::make_row_part(c->n);
    int64_t rc;
    const int nchunk = hd::ut_p_chunks(c->n, &rc);
    // columns come in powers of two >= 64; the largest that fits the budget
    const int64_t per_col = bytes_per_column(c, rk, nchunk, rp.nblk, o->top_k, o->k_y);
    int ldb = pow2_at_least(slots);
    if (hbm_budget_bytes > 0) {
        while (ldb > 64 && per_col * ldb > hbm_budget_bytes) ldb /= 2;
        if (per_col * ldb > hbm_budget_bytes)
            return fail(HD_ENOMEM, "hd_serve_open: budget %lld bytes is below one 64-column solve (%lld bytes)",
                        (long long)hbm_budget_bytes, (long long)(per_col * ldb));
        if (slots > ldb) slots = ldb;
    }
    Srv *v = new (std::nothrow) hd_server();
    if (!v) return fail(HD_ENOMEM, "hd_serve_open: out of host memory");
    hd_server *sv = static_cast<hd_server *>(v);
    v->c = c;
    v->o = *o;
    v->data = data_of(c);
    v->slots = slots;
    v->ldb = ldb;
    v->rk = rk;
    v->r_use = r_use;
    v->rp = rp;
    v->nchunk = nchunk;
    v->ticket.assign((size_t)ldb, -1);
    auto bail = [&](int code) {
        v->release();
        delete sv;
        return code;
    };
#define SRV_TRY(call)                                                                          \
    do {                                                                                       \
        hipError_t e_ = (call);                                                                \
        if (e_ != hipSuccess)                                                                  \
            return bail(fail(e_ == hipErrorOutOfMemory ? HD_ENOMEM : HD_EDEVICE, "%s: %s", #call, \
                             hipGetErrorString(e_)));                                          \
    } while (0)
    SRV_TRY(hipStreamCreate(&v->s));
    v->fused = c->u_mfma() && rk > 0;
    v->nrb = hd::uc_update_r_blocks(c->n);
    if (v->fused) SRV_TRY(v->Dg.ensure((size_t)rk * ldb * sizeof(double)));
    const size_t vec = (size_t)c->n * ldb * sizeof(float);
    SRV_TRY(v->X.ensure(vec));
    SRV_TRY(v->R.ensure(vec));
    SRV_TRY(v->P.ensure(vec));
    SRV_TRY(v->Q.ensure(vec));
    if (rk > 0) {
        if (!v->fused) SRV_TRY(v->Z.ensure(vec));
        SRV_TRY(v->Cpart.ensure((size_t)nchunk * rk * ldb * sizeof(float)));
        SRV_TRY(v->Cl.ensure((size_t)rk * ldb * sizeof(float)));
        SRV_TRY(v->Cs.ensure((size_t)rk * ldb * sizeof(float)));
        SRV_TRY(v->ClT.ensure((size_t)rk * ldb * 2 * sizeof(uint16_t)));
        if (c->u_mfma()) SRV_TRY(v->PT.ensure((size_t)ldb * c->ldut * 2 * sizeof(uint16_t)));
        SRV_TRY(v->csc.ensure((size_t)rk * ldb * sizeof(float)));
        SRV_TRY(v->cst.ensure((size_t)rk * ldb * 2 * sizeof(uint16_t)));
    }
    SRV_TRY(v->part.ensure((size_t)(v->fused && v->nrb > rp.nblk ? v->nrb : rp.nblk) * ldb * sizeof(double)));
    SRV_TRY(v->scal.ensure((size_t)ldb * (5 * sizeof(double) + 4 * sizeof(int32_t)) + 128 * sizeof(int32_t)));
    SRV_TRY(v->err.ensure(16));
    SRV_TRY(v->cols.ensure((size_t)2 * ldb * sizeof(int32_t)));  // admitted columns, then the ones to clear
    SRV_TRY(v->maxit.ensure((size_t)ldb * sizeof(int32_t)));
    SRV_TRY(v->xc.ensure(vec));
    SRV_TRY(v->xq.ensure((size_t)c->n * ldb * sizeof(float)));
    SRV_TRY(v->topk.ensure(hd::topk_scratch_bytes(ldb, c->n, o->top_k)));
    SRV_TRY(v->rids.ensure((size_t)ldb * o->top_k * sizeof(int32_t)));
    SRV_TRY(v->rsc.ensure((size_t)ldb * o->top_k * sizeof(float)));
    SRV_TRY(v->ybuf.ensure((size_t)ldb * o->k_y * (sizeof(int32_t) + sizeof(float))));
    void *hp = nullptr;
    SRV_TRY(hipHostMalloc(&hp, (3 * ldb + 16) * sizeof(int32_t), hipHostMallocDefault));
    v->h = reinterpret_cast<int32_t *>(hp);
    SRV_TRY(hipHostMalloc(&hp, ldb * sizeof(double), hipHostMallocDefault));
    v->hr = reinterpret_cast<double *>(hp);
    {
        char *b = v->scal.as<char>();
        hd::CgState &st = v->st;
        st.rho0 = reinterpret_cast<double *>(b); b += ldb * sizeof(double);
        st.rho = reinterpret_cast<double *>(b); b += ldb * sizeof(double);
        st.a = reinterpret_cast<double *>(b); b += ldb * sizeof(double);
        st.beta = reinterpret_cast<double *>(b); b += ldb * sizeof(double);
        st.relres = reinterpret_cast<double *>(b); b += ldb * sizeof(double);
        st.active = reinterpret_cast<int32_t *>(b); b += ldb * sizeof(int32_t);
        st.iters = reinterpret_cast<int32_t *>(b); b += ldb * sizeof(int32_t);
        st.status = reinterpret_cast<int32_t *>(b); b += ldb * sizeof(int32_t);
        st.maxit = reinterpret_cast<int32_t *>(b); b += ldb * sizeof(int32_t);
        st.nact_part = reinterpret_cast<int32_t *>(b);
    }
    // every column starts free: zero vectors, inactive, zero coefficients
    SRV_TRY(hd::launch_fill_zero(v->X.as<float>(), (size_t)c->n * ldb, v->s));
    SRV_TRY(hd::launch_fill_zero(v->R.as<float>(), (size_t)c->n * ldb, v->s));
    SRV_TRY(hd::launch_fill_zero(v->P.as<float>(), (size_t)c->n * ldb, v->s));
    SRV_TRY(hd::launch_fill_zero(v->scal.as<float>(), v->scal.bytes / sizeof(float), v->s));
    if (rk > 0) SRV_TRY(hd::launch_fill_zero(v->Cs.as<float>(), (size_t)rk * ldb, v->s));
    // the split P^T of the bfloat16 forms is kept equal to the split of P
    // from here on (admission writes the new columns' part, every iteration
    // the whole of it with the new P)
    if (v->fused) SRV_TRY(hd::launch_fill_zero(v->PT.as<float>(), (size_t)ldb * c->ldut, v->s));
    v->dirty.assign((size_t)ldb, 0);
    SRV_TRY(hipStreamSynchronize(v->s));
#undef SRV_TRY
    *out = sv;
    return HD_OK;
}

int64_t hd_serve_column_bytes(const hd_ctx *c, const hd_query_opts *o) {
    if (!c || !o || c->n == 0) return 0;
    const int r_use = o->rank_r < 0 ? c->r : (o->rank_r < c->r ? o->rank_r : c->r);
    const int rk = (r_use + 31) / 32 * 32;
    int64_t rc;
    const int nchunk = hd::ut_p_chunks(c->n, &rc);
    return bytes_per_column(c, rk, nchunk, hd::make_row_part(c->n).nblk, o->top_k, o->k_y);
}

int hd_serve_slots(const hd_server *v) { return v ? v->slots : 0; }

int hd_serve_in_use(const hd_server *v) {
    if (!v) return 0;
    int k = 0;
    for (int64_t t : v->ticket) k += t >= 0;
    return k;
}

int hd_serve_cancel(hd_server *v, int32_t n, const int64_t *tickets) {
    g_err.clear();
    if (!v) return fail(HD_EINVAL, "hd_serve_cancel: NULL server");
    if (n < 0 || (n > 0 && !tickets)) return fail(HD_EINVAL, "hd_serve_cancel: bad n or NULL tickets");
    hd_ctx *c = v->c;
    std::vector<int32_t> cols;
    for (int q = 0; q < n; ++q) {
        if (tickets[q] < 0) continue;
        for (int t = 0; t < v->ldb; ++t)
            if (v->ticket[(size_t)t] == tickets[q]) {
                bool seen = false;
                for (int32_t k : cols) seen = seen || k == t;
                if (!seen) cols.push_back(t);
            }
    }
    if (cols.empty()) return 0;
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = v->s;
    // after the queued steps on the server's stream: the columns stop and
    // leave; the other columns' arithmetic does not involve them
    HIP_TRY(hipMemcpyAsync(v->cols.p, cols.data(), cols.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hd::launch_cancel_cols(v->st, v->cols.as<int32_t>(), (int)cols.size(), s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int32_t t : cols) {
        v->ticket[(size_t)t] = -1;
        v->dirty[(size_t)t] = 1;
    }
    return (int)cols.size();
}

void hd_serve_close(hd_server *v) {
    if (!v) return;
    if (v->s) (void)hipStreamSynchronize(v->s);
    v->release();
    delete v;
}

int hd_serve_submit(hd_server *v, int32_t n, const float *q_desc, const int32_t *y_ids,
                    const float *y_val, const int32_t *max_iter, int64_t *tickets) {
    g_err.clear();
    if (!v) return fail(HD_EINVAL, "hd_serve_submit: NULL server");
    if (n < 0 || (n > 0 && !tickets)) return fail(HD_EINVAL, "hd_serve_submit: bad n or NULL tickets");
    hd_ctx *c = v->c;
    if (data_of(c) != v->data)
        return fail(HD_ESTATE, "%s: the context's data changed since the server was opened", "hd_serve_submit");
    const int ky = v->o.k_y, ldb = v->ldb;
    if (q_desc) {
        if (c->d == 0) return fail(HD_ESTATE, "hd_serve_submit: descriptors not loaded");
    } else if (n > 0 && (!y_ids || !y_val)) {
        return fail(HD_EINVAL, "hd_serve_submit: give q_desc or both y_ids and y_val");
    }
    std::vector<int32_t> freec;
    for (int t = 0; t < v->slots; ++t)
        if (v->ticket[(size_t)t] < 0) freec.push_back(t);
    const int m = n < (int)freec.size() ? n : (int)freec.size();
    if (m == 0) return 0;
    for (int t = 0; t < m && max_iter; ++t)
        if (max_iter[t] < 0) return fail(HD_EINVAL, "hd_serve_submit: max_iter[%d] < 0", t);
    // y ids are checked here, before any column changes
    for (size_t t = 0; !q_desc && t < (size_t)m * ky; ++t)
        if (y_ids[t] < 0 || (int64_t)y_ids[t] >= c->n)
            return fail(HD_EINVAL, "hd_serve_submit: y id %d of request %zu is outside [0, n)", y_ids[t], t / ky);
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = v->s;
    const int64_t N = c->n;
    int32_t *yi = v->ybuf.as<int32_t>();
    float *yv = reinterpret_cast<float *>(yi + (size_t)ldb * ky);
    if (q_desc) {
        // step 1 for the admitted queries: similarities, top-k_y, cube
        const int64_t lds = (N + 63) / 64 * 64;
        HIP_TRY(v->qbuf.ensure((size_t)m * c->d * sizeof(float)));
        HIP_TRY(v->sim.ensure((size_t)m * lds * sizeof(float)));
        HIP_TRY(v->topk.ensure(hd::topk_scratch_bytes(m > ldb ? m : ldb, N, ky > v->o.top_k ? ky : v->o.top_k)));
        HIP_TRY(hipMemcpyAsync(v->qbuf.p, q_desc, (size_t)m * c->d * sizeof(float), hipMemcpyHostToDevice, s));
        if (c->v_dtype != HD_F32) {
            HIP_TRY(v->qsplit.ensure((size_t)2 * hd::sim_qsplit_rows(m) * c->ldv * sizeof(uint16_t)));
            HIP_TRY(hd::launch_sim_bf16(N, m, c->d, v->qbuf.as<float>(), c->Vb.p, c->ldv, v->qsplit.as<uint16_t>(),
                                        v->sim.as<float>(), lds, s, c->v_scale()));
        } else {
            HIP_TRY(hd::launch_sim(N, m, c->d, v->qbuf.as<float>(), c->V.as<float>(), c->ldv,
                                   v->sim.as<float>(), lds, s));
        }
        HIP_TRY(hd::launch_topk(m, N, v->sim.as<float>(), lds, ky, v->topk.p, yi, yv, 1, s));
    } else {
        HIP_TRY(hipMemcpyAsync(yi, y_ids, (size_t)m * ky * sizeof(int32_t), hipMemcpyHostToDevice, s));
        HIP_TRY(hipMemcpyAsync(yv, y_val, (size_t)m * ky * sizeof(float), hipMemcpyHostToDevice, s));
    }
    std::vector<int32_t> caps((size_t)m);
    for (int t = 0; t < m; ++t) caps[(size_t)t] = max_iter ? max_iter[t] : v->o.max_iter;
    // the admitted columns, then those of them to clear first: all of them
    // without the bfloat16 forms, else the dirty ones
    std::vector<int32_t> lists(freec.begin(), freec.begin() + m);
    for (int t = 0; t < m; ++t)
        if (!v->fused || v->dirty[(size_t)freec[(size_t)t]]) lists.push_back(freec[(size_t)t]);
    const int nz = (int)lists.size() - m;
    HIP_TRY(hipMemcpyAsync(v->cols.p, lists.data(), lists.size() * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(v->maxit.p, caps.data(), (size_t)m * sizeof(int32_t), hipMemcpyHostToDevice, s));
    const int32_t *cols = v->cols.as<int32_t>(), *zcols = cols + m;
    HIP_TRY(hd::launch_fill_zero(v->err.as<float>(), 1, s));
    HIP_TRY(hd::launch_zero_cols(N, ldb, v->X.as<float>(), v->R.as<float>(), v->P.as<float>(), zcols, nz, s));
    HIP_TRY(hd::launch_scatter_y(m, ky, yi, yv, N, ldb, v->R.as<float>(), v->P.as<float>(),
                                 v->err.as<int32_t>(), s, cols));
    if (v->fused) {
        uint16_t *PTh = v->PT.as<uint16_t>(), *PTl = PTh + (size_t)ldb * c->ldut;
        HIP_TRY(hd::launch_pt_admit(m, ky, yi, cols, zcols, nz, N, ldb, v->P.as<float>(), c->ldut, PTh, PTl, s));
    }
    for (int t = 0; t < m; ++t) v->dirty[(size_t)freec[(size_t)t]] = 1;
    HIP_TRY(hd::launch_ynorm_part(m, ky, yi, N, ldb, v->R.as<float>(), v->part.as<double>(), s, cols));
    HIP_TRY(hd::launch_init_cols(ldb, v->part.as<double>(), 1, v->st, cols, v->maxit.as<int32_t>(), m, s));
    if (v->rk > 0) {
        const bool ubf = c->u_mfma();
        HIP_TRY(hd::launch_gather_proj(m, ky, yi, yv, N, ubf ? c->Ub.p : c->U.p, c->ub_lo(), c->u_fmt(), c->rp,
                                       v->rk, v->r_use, c->lam.as<double>(), v->o.alpha, ldb, v->Cs.as<float>(),
                                       nullptr, s, cols, nullptr, nullptr, c->u_scale()));
    }
    HIP_TRY(hipMemcpyAsync(v->h + 3 * ldb, v->err.p, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (v->h[3 * ldb] != 0) {
        // undo: stop the columns just started; they stay free (their state is
        // reset on the next admission)
        HIP_TRY(hd::launch_cancel_cols(v->st, cols, m, s));
        HIP_TRY(hipStreamSynchronize(s));
        return fail(HD_EINVAL, "hd_serve_submit: a y id is outside [0, n)");
    }
    for (int t = 0; t < m; ++t) {
        v->ticket[(size_t)freec[(size_t)t]] = v->next_ticket;
        tickets[t] = v->next_ticket++;
    }
    return m;
}

int hd_serve_step(hd_server *v, int32_t iters) {
    g_err.clear();
    if (!v) return fail(HD_EINVAL, "hd_serve_step: NULL server");
    if (iters < 0) return fail(HD_EINVAL, "hd_serve_step: iters < 0");
    hd_ctx *c = v->c;
    if (data_of(c) != v->data)
        return fail(HD_ESTATE, "%s: the context's data changed since the server was opened", "hd_serve_step");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = v->s;
    const int64_t N = c->n;
    const int ldb = v->ldb, rk = v->rk;
    const bool ubf = c->u_mfma();
    const hd::IterGuard g{nullptr, 0};
    float *X = v->X.as<float>(), *R = v->R.as<float>(), *P = v->P.as<float>(), *Q = v->Q.as<float>();
    uint16_t *ClT_hi = v->ClT.as<uint16_t>(), *ClT_lo = ClT_hi ? ClT_hi + (size_t)rk * ldb : nullptr;
    // Free columns are never active and admission fills the lowest free ones,
    // so the bfloat16 iteration runs its wide kernels over the occupied
    // prefix only: columns [0, w), w the highest occupied column + 1 rounded
    // up to 64 (row stride stays ldb). Each column's arithmetic does not
    // depend on w; the scalar steps run over all columns (the free ones are
    // inactive and keep their state).
    int hi = -1;
    for (int t = 0; t < ldb; ++t)
        if (v->ticket[(size_t)t] >= 0) hi = t;
    const int w = hi < 0 ? 0 : (hi + 64) / 64 * 64;
    for (int it = 0; it < iters && v->fused && w > 0; ++it) {
        // L1 U1^T P for every column (a newly admitted column has P = y),
        // from the split P^T that admission and the previous x/p update
        // wrote; the correction goes into the residual update
        uint16_t *PTh = v->PT.as<uint16_t>(), *PTl = PTh + (size_t)ldb * c->ldut;
        HIP_TRY(hd::launch_ut_p_bf16(N, c->u_comp(), c->ldut, rk, PTh, PTl, ldb,
                                     v->Cpart.as<float>(), g, s, c->tv(HD_TUNE_UTP_NT, w), w));
        HIP_TRY(hd::launch_reduce_c(v->nchunk, v->Cpart.as<float>(), rk, ldb, c->lam.as<double>(), v->r_use,
                                    v->Cl.as<float>(), g, s, v->Dg.as<double>(), v->o.alpha, c->u_scale()));
        HIP_TRY(hd::launch_split_t(v->Cl.as<float>(), rk, ldb, ClT_hi, ClT_lo, g, s));
        HIP_TRY(hd::launch_spmm(N, c->rowptr.as<int64_t>(), c->col.as<int32_t>(), c->val.as<float>(), P, P, Q,
                                ldb, v->o.alpha, v->rp, v->part.as<double>(), g, s, c->tv(HD_TUNE_SPMM_CPL, w),
                                w, nullptr, c->bands(), c->cuts()));
        HIP_TRY(hd::launch_cg_step_a(ldb, v->part.as<double>(), v->rp.nblk, v->st, g, s, v->Dg.as<double>(), rk));
        HIP_TRY(hd::launch_uc_update_r_bf16(N, c->u_item(), c->rp, rk, ClT_hi, ClT_lo, ldb, Q,
                                            v->o.alpha, R, v->st.a, v->part.as<double>(), g, s,
                                            c->tv(HD_TUNE_UC_NT, w), w, nullptr, v->st.iters, v->st.maxit));
        HIP_TRY(hd::launch_cg_step_b(ldb, v->part.as<double>(), v->nrb, v->o.tol, v->st, g, v->st.nact_part, s));
        HIP_TRY(hd::launch_update_xp_pt(N, ldb, X, P, R, v->st.a, v->st.beta, v->st.active, c->ldut, PTh, PTl, g, s,
                                        nullptr, w, v->st.iters));
    }
    // every column below w went through the x/p update: a stopped one is clear
    if (v->fused && iters > 0)
        for (int t = 0; t < w; ++t) v->dirty[(size_t)t] = 0;
    for (int it = 0; it < iters && !v->fused; ++it) {
        const float *Zs = P;
        if (rk > 0) {
            // L1 U1^T P for every column (a newly admitted column has P = y)
            if (ubf) {
                uint16_t *PTh = v->PT.as<uint16_t>(), *PTl = PTh + (size_t)ldb * c->ldut;
                HIP_TRY(hd::launch_split_pt(N, ldb, P, c->ldut, PTh, PTl, g, s));
                HIP_TRY(hd::launch_ut_p_bf16(N, c->u_comp(), c->ldut, rk, PTh, PTl, ldb,
                                             v->Cpart.as<float>(), g, s, c->tv(HD_TUNE_UTP_NT, ldb)));
            } else {
                HIP_TRY(hd::launch_ut_p(N, c->U.as<float>(), c->rp, rk, P, ldb, v->Cpart.as<float>(), g, s));
            }
            HIP_TRY(hd::launch_reduce_c(v->nchunk, v->Cpart.as<float>(), rk, ldb, c->lam.as<double>(), v->r_use,
                                        v->Cl.as<float>(), g, s, nullptr, 0.0, c->u_scale()));
            if (ubf) {
                HIP_TRY(hd::launch_split_t(v->Cl.as<float>(), rk, ldb, ClT_hi, ClT_lo, g, s));
                HIP_TRY(hd::launch_u_c_bf16(N, c->u_item(), c->rp, rk, ClT_hi, ClT_lo, ldb, P, v->o.alpha,
                                            v->Z.as<float>(), g, s, c->tv(HD_TUNE_UC_NT, ldb)));
            } else {
                HIP_TRY(hd::launch_u_c(N, c->U.as<float>(), c->rp, rk, v->Cl.as<float>(), ldb, P, v->o.alpha,
                                       v->Z.as<float>(), g, s));
            }
            Zs = v->Z.as<float>();
        }
        HIP_TRY(hd::launch_spmm(N, c->rowptr.as<int64_t>(), c->col.as<int32_t>(), c->val.as<float>(), P, Zs, Q,
                                ldb, v->o.alpha, v->rp, v->part.as<double>(), g, s, c->tv(HD_TUNE_SPMM_CPL, ldb),
                                0, nullptr, c->bands(), c->cuts()));
        HIP_TRY(hd::launch_cg_step_a(ldb, v->part.as<double>(), v->rp.nblk, v->st, g, s));
        HIP_TRY(hd::launch_update_r(N, ldb, Q, R, v->rp, v->st.a, v->part.as<double>(), g, s));
        HIP_TRY(hd::launch_cg_step_b(ldb, v->part.as<double>(), v->rp.nblk, v->o.tol, v->st, g,
                                     v->st.nact_part, s));
        HIP_TRY(hd::launch_update_xp(N, ldb, X, P, R, v->st.a, v->st.beta, v->st.active, g, s));
    }
    return HD_OK;
}

int hd_serve_poll(hd_server *v, int32_t max_out, int64_t *tickets, int32_t *ids, float *scores,
                  int32_t *iters, double *relres, int32_t *status) {
    g_err.clear();
    if (!v) return fail(HD_EINVAL, "hd_serve_poll: NULL server");
    if (max_out < 0 || (max_out > 0 && !tickets)) return fail(HD_EINVAL, "hd_serve_poll: bad max_out or NULL tickets");
    hd_ctx *c = v->c;
    if (data_of(c) != v->data)
        return fail(HD_ESTATE, "%s: the context's data changed since the server was opened", "hd_serve_poll");
    HIP_TRY(hipSetDevice(c->device));
    hipStream_t s = v->s;
    const int64_t N = c->n;
    const int ldb = v->ldb, rk = v->rk, K = v->o.top_k;
    HIP_TRY(hd::launch_cg_final(ldb, v->st, s));
    HIP_TRY(hipMemcpyAsync(v->h, v->st.active, ldb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(v->h + ldb, v->st.iters, ldb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(v->h + 2 * ldb, v->st.status, ldb * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(v->hr, v->st.relres, ldb * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    std::vector<int32_t> done;
    for (int t = 0; t < ldb && (int)done.size() < max_out; ++t)
        if (v->ticket[(size_t)t] >= 0 && v->h[t] == 0) done.push_back(t);
    const int m = (int)done.size();
    if (m == 0) return 0;
    const int ldc = pow2_at_least(m);
    HIP_TRY(hipMemcpyAsync(v->cols.p, done.data(), (size_t)m * sizeof(int32_t), hipMemcpyHostToDevice, s));
    HIP_TRY(hd::launch_gather_cols(N, ldb, v->X.as<float>(), v->Cs.as<float>(), rk, v->cols.as<int32_t>(), m,
                                   ldc, v->xc.as<float>(), v->csc.as<float>(), s, v->st.iters));
    float *xq = v->xq.as<float>();
    if (rk > 0 && c->u_mfma()) {
        uint16_t *hi = v->cst.as<uint16_t>(), *lo = hi + (size_t)rk * ldc;
        HIP_TRY(hd::launch_split_t(v->csc.as<float>(), rk, ldc, hi, lo, hd::IterGuard{nullptr, 0}, s));
        HIP_TRY(hd::launch_combine_bf16(N, m, c->u_item(), c->rp, rk, hi, lo, ldc, v->xc.as<float>(), xq,
                                        N, s, c->tv(HD_TUNE_UC_NT, ldc)));
    } else {
        HIP_TRY(hd::launch_combine(N, m, c->U.as<float>(), c->rp, rk, v->csc.as<float>(), ldc, v->xc.as<float>(),
                                   xq, N, s));
    }
    HIP_TRY(hd::launch_topk(m, N, xq, N, K, v->topk.p, v->rids.as<int32_t>(), v->rsc.as<float>(), 0, s));
    if (ids) HIP_TRY(hipMemcpyAsync(ids, v->rids.p, (size_t)m * K * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (scores) HIP_TRY(hipMemcpyAsync(scores, v->rsc.p, (size_t)m * K * sizeof(float), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    for (int t = 0; t < m; ++t) {
        const int col = done[(size_t)t];
        tickets[t] = v->ticket[(size_t)col];
        if (iters) iters[t] = v->h[ldb + col];
        if (status) status[t] = v->h[2 * ldb + col];
        if (relres) relres[t] = v->hr[col];
        v->ticket[(size_t)col] = -1;
    }
    return m;
}

}  // extern "C"
