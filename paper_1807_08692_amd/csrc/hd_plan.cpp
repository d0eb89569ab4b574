// Query plans: the query path captured into a HIP graph for a fixed batch
// size and replayed per batch (the batching form of the library).
//
// Capture reuses the same queueing code as hd_query_batch in its graph form
// (every CG iteration queued, device-side guards instead of host checks). A
// dry run queues the path once eagerly first, so every workspace buffer has
// its final size before capture and no allocation happens inside it. The
// graph bakes in buffer addresses, launch parameters and data layouts, so the
// plan snapshots them and captures again when any has changed.
#include "hd_internal.h"

#include <vector>

struct hd_plan {
    hd_ctx *c = nullptr;
    int B = 0, input = HD_PLAN_DESCRIPTORS;
    hd_query_opts o{};
    DevBuf q, yi, yv, rid, rsc;
    hipStream_t cs = nullptr;  // capture stream
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<intptr_t> snap;
    hd::CgState st{};  // the column state layout the graph was captured with

    void drop_graph() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        exec = nullptr;
        graph = nullptr;
    }
};

namespace {

std::vector<intptr_t> snapshot(const hd_ctx *c) {
    const DevBuf *bufs[] = {&c->rowptr, &c->col, &c->val, &c->cut, &c->U,    &c->Ub,   &c->UbT,  &c->lam,
                            &c->V,      &c->Vb,  &c->X,   &c->R,    &c->P,    &c->Q,    &c->Z,
                            &c->Cpart,  &c->Cl,  &c->Cs,  &c->ClT,  &c->CsT,  &c->PT,   &c->part,
                            &c->scal,   &c->xbuf, &c->sim, &c->ybuf, &c->topk, &c->err, &c->qsplit,
                            &c->Usr,    &c->Usc, &c->Usv, &c->Ustp, &c->Ustr, &c->Ustv, &c->Dg,
                            &c->ymask,  &c->uscale, &c->vscale, &c->pbar, &c->pre, &c->Vsm, &c->Usm,
                            &c->tsx};
    std::vector<intptr_t> v;
    for (const DevBuf *b : bufs) v.push_back((intptr_t)b->p);
    const int64_t meta[] = {c->n, c->nnz, c->r, c->rp, c->u_dtype, c->ldut, c->d, c->ldv, c->v_dtype};
    for (int64_t m : meta) v.push_back((intptr_t)m);
    for (int t : c->tune) v.push_back(t);
    v.push_back(c->persist_mode);
    v.push_back((intptr_t)c->persist_spin);
    return v;
}

int queue_plan(hd_plan *p) {
    const bool desc = p->input == HD_PLAN_DESCRIPTORS;
    return queue_query(p->c, p->B, desc ? p->q.as<float>() : nullptr, desc ? nullptr : p->yi.as<int32_t>(),
                       desc ? nullptr : p->yv.as<float>(), &p->o, p->rid.as<int32_t>(), p->rsc.as<float>(),
                       nullptr, nullptr, nullptr, p->cs, true, nullptr);
}

int capture(hd_plan *p) {
    hd_ctx *c = p->c;
    p->drop_graph();
    const bool timing = c->timing.on;
    c->timing.on = false;
    // dry run: brings every workspace buffer to its size for this plan
    int e = queue_plan(p);
    if (e == HD_OK && hipStreamSynchronize(p->cs) != hipSuccess) e = fail(HD_EDEVICE, "hd_plan: dry run failed");
    if (e == HD_OK) {
        hipError_t he = hipStreamBeginCapture(p->cs, hipStreamCaptureModeThreadLocal);
        if (he != hipSuccess) {
            e = fail(HD_EDEVICE, "hd_plan: begin capture: %s", hipGetErrorString(he));
        } else {
            e = queue_plan(p);
            hipGraph_t g = nullptr;
            he = hipStreamEndCapture(p->cs, &g);
            if (e == HD_OK && he != hipSuccess) e = fail(HD_EDEVICE, "hd_plan: end capture: %s", hipGetErrorString(he));
            if (e == HD_OK) {
                p->graph = g;
                he = hipGraphInstantiate(&p->exec, g, nullptr, nullptr, 0);
                if (he != hipSuccess) e = fail(HD_EDEVICE, "hd_plan: instantiate: %s", hipGetErrorString(he));
            } else if (g) {
                (void)hipGraphDestroy(g);
            }
        }
    }
    c->timing.on = timing;
    if (e != HD_OK) {
        p->drop_graph();
        return e;
    }
    p->snap = snapshot(c);
    p->st = c->st;
    return HD_OK;
}

}  // namespace

extern "C" {

int hd_plan_create(hd_ctx *c, int32_t B, int32_t input, const hd_query_opts *o, hd_plan **out) {
    g_err.clear();
    if (!out) return fail(HD_EINVAL, "hd_plan_create: out is NULL");
    *out = nullptr;
    if (!c) return fail(HD_EINVAL, "hd_plan_create: NULL context");
    if (!o) return fail(HD_EINVAL, "hd_plan_create: NULL options");
    if (input != HD_PLAN_DESCRIPTORS && input != HD_PLAN_Y)
        return fail(HD_EINVAL, "hd_plan_create: input kind %d unknown", input);
    if (c->n == 0) return fail(HD_ESTATE, "hd_plan_create: no graph loaded");
    if (B < 1 || B > 1024) return fail(HD_EINVAL, "hd_plan_create: B=%d not in [1, 1024]", B);
    if (o->top_k < 1) return fail(HD_EINVAL, "hd_plan_create: top_k must be >= 1");
    if (input == HD_PLAN_DESCRIPTORS && c->d == 0) return fail(HD_ESTATE, "hd_plan_create: descriptors not loaded");
    if (o->k_y < 1 || o->k_y > c->n || o->k_y > hd::kTopkMax)
        return fail(HD_EINVAL, "hd_plan_create: k_y=%d out of range", o->k_y);
    HIP_TRY(hipSetDevice(c->device));
    hd_plan *p = new (std::nothrow) hd_plan();
    if (!p) return fail(HD_ENOMEM, "hd_plan_create: out of host memory");
    p->c = c;
    p->B = B;
    p->input = input;
    p->o = *o;
    int e = HD_OK;
#define PLAN_TRY(x)                                                                              \
    do {                                                                                         \
        hipError_t e_ = (x);                                                                     \
        if (e_ != hipSuccess && e == HD_OK) e = fail(HD_EDEVICE, "hd_plan_create: %s", hipGetErrorString(e_)); \
    } while (0)
    PLAN_TRY(hipStreamCreate(&p->cs));
    if (input == HD_PLAN_DESCRIPTORS) {
        PLAN_TRY(p->q.ensure((size_t)B * c->d * sizeof(float)));
        if (e == HD_OK) PLAN_TRY(hd::launch_fill_zero(p->q.as<float>(), (size_t)B * c->d, p->cs));
    } else {
        PLAN_TRY(p->yi.ensure((size_t)B * o->k_y * sizeof(int32_t)));
        PLAN_TRY(p->yv.ensure((size_t)B * o->k_y * sizeof(float)));
        if (e == HD_OK) PLAN_TRY(hd::launch_fill_zero(p->yi.as<float>(), (size_t)B * o->k_y, p->cs));
        if (e == HD_OK) PLAN_TRY(hd::launch_fill_zero(p->yv.as<float>(), (size_t)B * o->k_y, p->cs));
    }
    PLAN_TRY(p->rid.ensure((size_t)B * o->top_k * sizeof(int32_t)));
    PLAN_TRY(p->rsc.ensure((size_t)B * o->top_k * sizeof(float)));
#undef PLAN_TRY
    if (e == HD_OK) e = capture(p);
    if (e != HD_OK) {
        hd_plan_destroy(p);
        return e;
    }
    *out = p;
    return HD_OK;
}

int hd_plan_run(hd_plan *p, const float *q_desc, const int32_t *y_ids, const float *y_val,
                int32_t *rank_ids, float *rank_scores, int32_t *iters, double *relres,
                int32_t *status, void *stream) {
    g_err.clear();
    if (!p) return fail(HD_EINVAL, "hd_plan_run: NULL plan");
    hd_ctx *c = p->c;
    const bool desc = p->input == HD_PLAN_DESCRIPTORS;
    if (desc ? !q_desc : (!y_ids || !y_val)) return fail(HD_EINVAL, "hd_plan_run: missing input");
    HIP_TRY(hipSetDevice(c->device));
    if (!p->exec || snapshot(c) != p->snap) {
        const int e = capture(p);
        if (e != HD_OK) return e;
    }
    hipStream_t s = (hipStream_t)stream;
    const int B = p->B, ky = p->o.k_y, K = p->o.top_k;
    if (desc) {
        HIP_TRY(hipMemcpyAsync(p->q.p, q_desc, (size_t)B * c->d * sizeof(float), hipMemcpyDeviceToDevice, s));
    } else {
        HIP_TRY(hipMemcpyAsync(p->yi.p, y_ids, (size_t)B * ky * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
        HIP_TRY(hipMemcpyAsync(p->yv.p, y_val, (size_t)B * ky * sizeof(float), hipMemcpyDeviceToDevice, s));
    }
    HIP_TRY(hipGraphLaunch(p->exec, s));
    if (rank_ids)
        HIP_TRY(hipMemcpyAsync(rank_ids, p->rid.p, (size_t)B * K * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    if (rank_scores)
        HIP_TRY(hipMemcpyAsync(rank_scores, p->rsc.p, (size_t)B * K * sizeof(float), hipMemcpyDeviceToDevice, s));
    // the plan's own copy: later calls with another width re-carve c->st
    const hd::CgState &st = p->st;
    if (iters) HIP_TRY(hipMemcpyAsync(iters, st.iters, B * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (status) HIP_TRY(hipMemcpyAsync(status, st.status, B * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (relres) HIP_TRY(hipMemcpyAsync(relres, st.relres, B * sizeof(double), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipMemcpyAsync(c->h_pinned + 200, c->err.p, 2 * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    if (c->h_pinned[200] != 0) return fail(HD_EINVAL, "hd_plan_run: a y id is outside [0, n)");
    if (c->h_pinned[201] != 0)
        return fail(HD_EDEVICE, "hd_plan_run: a grid barrier wait of the persistent CG ran past its limit");
    return HD_OK;
}

void hd_plan_destroy(hd_plan *p) {
    if (!p) return;
    if (p->c) (void)hipSetDevice(p->c->device);
    if (p->cs) (void)hipStreamSynchronize(p->cs);
    p->drop_graph();
    DevBuf *bufs[] = {&p->q, &p->yi, &p->yv, &p->rid, &p->rsc};
    for (DevBuf *b : bufs) b->release();
    if (p->cs) (void)hipStreamDestroy(p->cs);
    delete p;
}

}  // extern "C"
