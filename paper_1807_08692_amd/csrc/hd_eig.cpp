// On-device top-r eigensolver: the r algebraically largest eigenpairs of the
// loaded S, which the hybrid method takes as its off-line input (Section
// 4.1, eq. (w-decomp)), computed by Chebyshev-filtered subspace iteration in
// double precision on a block of m >= r vectors:
//   1. Rayleigh-Ritz: SX = S X, H = X^T S X, H = Z W Z^T, X <- X Z, SX <- SX Z;
//   2. stop when the r leading residuals ||S x_j - w_j x_j|| are below tol
//      (or at the iteration or time limit);
//   3. filter: X <- T_d((S - c)/e) X with the Chebyshev polynomial of degree d
//      that damps [lambda_min, w_m] (c, e its centre and half-width), by the
//      three-term recurrence;
//   4. orthonormalise X by shifted CholeskyQR (one shifted pass, then two
//      plain passes; Fukaya et al. 2020), and go to 1.
// The sparse products, the recurrence and every product over the N rows of a
// block (Gram matrices, X^T S X, the rotations X Z and X R^-1) run in this
// library's kernels (k_eig.hip, k_eig_gemm.hip: FP64 matrix cores). Only the
// m x m steps use rocSOLVER: the Cholesky factor and its inverse, and the
// m x m symmetric eigenproblem. Blocks are item-major N x m; the m x m
// matrices handed to rocSOLVER are column-major.
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <vector>

#include "hd_internal.h"

namespace {

struct Blas {
    rocblas_handle h = nullptr;
    ~Blas() {
        if (h) (void)rocblas_destroy_handle(h);
    }
};

#define RB_TRY(x)                                                                              \
    do {                                                                                       \
        rocblas_status st_ = (x);                                                              \
        if (st_ != rocblas_status_success)                                                     \
            return fail(HD_EDEVICE, "hd_compute_eigs: %s failed (%d)", #x, (int)st_);          \
    } while (0)

}  // namespace

extern "C" {

int hd_compute_eigs(hd_ctx *c, int32_t r, int32_t dtype, const hd_eig_opts *opts, double *lambda_out,
                    double *resid_out, float *U_out) {
    g_err.clear();
    if (!c) return fail(HD_EINVAL, "hd_compute_eigs: NULL context");
    if (c->n == 0) return fail(HD_ESTATE, "hd_compute_eigs: no graph loaded");
    if (!opts) return fail(HD_EINVAL, "hd_compute_eigs: NULL options");
    const int64_t N = c->n;
    const int m = (int)(((int64_t)r + std::max(opts->guard, 1) + 63) / 64 * 64);
    if (r < 1 || m > N) return fail(HD_EINVAL, "hd_compute_eigs: r=%d with its guard exceeds n", r);
    if (opts->degree < 1 || opts->degree > 64) return fail(HD_EINVAL, "hd_compute_eigs: degree not in [1, 64]");
    if (opts->max_outer < 1) return fail(HD_EINVAL, "hd_compute_eigs: max_outer < 1");
    if (!(opts->lambda_min >= -1.0 - 1e-12 && opts->lambda_min < 1.0))
        return fail(HD_EINVAL, "hd_compute_eigs: lambda_min not in [-1, 1)");
    if (dtype != HD_F32 && dtype != HD_BF16 && dtype != HD_BF16X2)
        return fail(HD_EINVAL, "hd_compute_eigs: dtype %d not supported", dtype);
    HIP_TRY(hipSetDevice(c->device));
    const auto t0 = std::chrono::steady_clock::now();
    const size_t blk = (size_t)N * m * sizeof(double);
    DevBuf X, SX, T1, T2, G, W, Wk, info, part, Gpart;
    HIP_TRY(X.ensure(blk));
    HIP_TRY(SX.ensure(blk));
    HIP_TRY(T1.ensure(blk));
    HIP_TRY(T2.ensure(blk));
    HIP_TRY(G.ensure((size_t)m * m * sizeof(double)));
    HIP_TRY(W.ensure((size_t)m * sizeof(double)));
    HIP_TRY(Wk.ensure((size_t)m * sizeof(double)));
    HIP_TRY(info.ensure(sizeof(rocblas_int)));
    HIP_TRY(Gpart.ensure((size_t)hd::gram_chunks(N) * m * m * sizeof(double)));
    const int64_t rb = std::max<int64_t>(1024, (N + 1023) / 1024);
    const int nblk = (int)((N + rb - 1) / rb);
    HIP_TRY(part.ensure((size_t)nblk * m * sizeof(double)));
    hipStream_t s = nullptr;
    Blas bl;
    RB_TRY(rocblas_create_handle(&bl.h));
    RB_TRY(rocblas_set_stream(bl.h, s));
    const int64_t *rowptr = c->rowptr.as<int64_t>();
    const int32_t *col = c->col.as<int32_t>();
    const float *val = c->val.as<float>();
    double *x = X.as<double>(), *sx = SX.as<double>(), *t1 = T1.as<double>(), *t2 = T2.as<double>();
    std::vector<double> hG((size_t)m * m), w(m), res(m);

    // orthonormalise the block held in px (shifted CholeskyQR3): G = X^T X,
    // G + shift = R^T R (Cholesky), X <- X R^-1 out of place into ptmp, then
    // the two pointers swap
    auto orth = [&](double *&px, double *&ptmp) -> int {
        double shift = 0.0;
        for (int pass = 0; pass < 3; ++pass) {
            for (int attempt = 0;; ++attempt) {
                HIP_TRY(hd::launch_gram(N, m, px, px, Gpart.as<double>(), G.as<double>(), s));
                HIP_TRY(hipMemcpy(hG.data(), G.p, hG.size() * sizeof(double), hipMemcpyDeviceToHost));
                if (pass == 0 || attempt > 0) {
                    double tr = 0.0;
                    for (int j = 0; j < m; ++j) tr += hG[(size_t)j * m + j];
                    const double base = 11.0 * ((double)m * N + (double)m * (m + 1)) * 1.1102230246251565e-16 * tr;
                    shift = attempt == 0 ? base : shift * 10.0;
                    for (int j = 0; j < m; ++j) hG[(size_t)j * m + j] += shift;
                    HIP_TRY(hipMemcpy(G.p, hG.data(), hG.size() * sizeof(double), hipMemcpyHostToDevice));
                }
                RB_TRY(rocsolver_dpotrf(bl.h, rocblas_fill_upper, m, G.as<double>(), m, info.as<rocblas_int>()));
                rocblas_int inf = 0;
                HIP_TRY(hipMemcpy(&inf, info.p, sizeof(inf), hipMemcpyDeviceToHost));
                if (inf == 0) break;
                if (attempt >= 6) return fail(HD_EDEVICE, "hd_compute_eigs: Cholesky of the Gram matrix failed");
            }
            // R^-1 (upper, column-major), its strict lower part zeroed, then
            // X <- X R^-1 (item-major: row i of X times R^-1)
            RB_TRY(rocsolver_dtrtri(bl.h, rocblas_fill_upper, rocblas_diagonal_non_unit, m, G.as<double>(), m,
                                    info.as<rocblas_int>()));
            rocblas_int inf = 0;
            HIP_TRY(hipMemcpy(&inf, info.p, sizeof(inf), hipMemcpyDeviceToHost));
            if (inf != 0) return fail(HD_EDEVICE, "hd_compute_eigs: inverse of the Cholesky factor failed");
            HIP_TRY(hipMemcpy(hG.data(), G.p, hG.size() * sizeof(double), hipMemcpyDeviceToHost));
            for (int q = 0; q < m; ++q)
                for (int p = q + 1; p < m; ++p) hG[(size_t)q * m + p] = 0.0;
            HIP_TRY(hipMemcpy(G.p, hG.data(), hG.size() * sizeof(double), hipMemcpyHostToDevice));
            HIP_TRY(hd::launch_rotate(N, m, px, G.as<double>(), m, ptmp, s));
            std::swap(px, ptmp);
        }
        return HD_OK;
    };

    HIP_TRY(hd::launch_eig_rand(N, m, opts->seed, x, s));
    int e = orth(x, t1);
    if (e != HD_OK) return e;
    int outer = 0;
    double maxres = 0.0;
    for (;; ++outer) {
        // Rayleigh-Ritz
        HIP_TRY(hd::launch_eig_cheb(N, rowptr, col, val, m, x, nullptr, sx, 1.0, 0.0, 0.0, s));
        HIP_TRY(hd::launch_gram(N, m, x, sx, Gpart.as<double>(), G.as<double>(), s));
        HIP_TRY(hipMemcpy(hG.data(), G.p, hG.size() * sizeof(double), hipMemcpyDeviceToHost));
        for (int a = 0; a < m; ++a)
            for (int b = a + 1; b < m; ++b) {
                const double v = 0.5 * (hG[(size_t)a * m + b] + hG[(size_t)b * m + a]);
                hG[(size_t)a * m + b] = hG[(size_t)b * m + a] = v;
            }
        HIP_TRY(hipMemcpy(G.p, hG.data(), hG.size() * sizeof(double), hipMemcpyHostToDevice));
        RB_TRY(rocsolver_dsyevd(bl.h, rocblas_evect_original, rocblas_fill_upper, m, G.as<double>(), m, W.as<double>(),
                                Wk.as<double>(), info.as<rocblas_int>()));
        rocblas_int inf = 0;
        HIP_TRY(hipMemcpy(&inf, info.p, sizeof(inf), hipMemcpyDeviceToHost));
        if (inf != 0) return fail(HD_EDEVICE, "hd_compute_eigs: Rayleigh-Ritz eigensolve failed (%d)", (int)inf);
        // descending order: reverse the eigenvector columns
        std::vector<double> wa(m);
        HIP_TRY(hipMemcpy(wa.data(), W.p, m * sizeof(double), hipMemcpyDeviceToHost));
        HIP_TRY(hipMemcpy(hG.data(), G.p, hG.size() * sizeof(double), hipMemcpyDeviceToHost));
        std::vector<double> Z((size_t)m * m);
        for (int j = 0; j < m; ++j) {
            w[j] = wa[m - 1 - j];
            std::copy(hG.begin() + (size_t)(m - 1 - j) * m, hG.begin() + (size_t)(m - j) * m, Z.begin() + (size_t)j * m);
        }
        HIP_TRY(hipMemcpy(G.p, Z.data(), Z.size() * sizeof(double), hipMemcpyHostToDevice));
        HIP_TRY(hipMemcpy(W.p, w.data(), m * sizeof(double), hipMemcpyHostToDevice));
        // X <- X Z, SX <- SX Z (column-major: Z^T X)
        HIP_TRY(hd::launch_rotate(N, m, x, G.as<double>(), m, t1, s));
        HIP_TRY(hd::launch_rotate(N, m, sx, G.as<double>(), m, t2, s));
        std::swap(x, t1);
        std::swap(sx, t2);
        // residuals
        HIP_TRY(hd::launch_eig_resid(N, m, sx, x, W.as<double>(), rb, nblk, part.as<double>(), s));
        std::vector<double> hp((size_t)nblk * m);
        HIP_TRY(hipMemcpy(hp.data(), part.p, hp.size() * sizeof(double), hipMemcpyDeviceToHost));
        maxres = 0.0;
        for (int j = 0; j < m; ++j) {
            double acc = 0.0;
            for (int b = 0; b < nblk; ++b) acc += hp[(size_t)b * m + j];
            res[j] = std::sqrt(acc);
            if (j < r) maxres = std::max(maxres, res[j]);
        }
        const double secs = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        if (maxres <= opts->tol || outer + 1 >= opts->max_outer ||
            (opts->time_budget_s > 0 && secs >= opts->time_budget_s))
            break;
        // Chebyshev filter on [lambda_min, w_m]
        const double a = opts->lambda_min, b = w[m - 1];
        const double cc = 0.5 * (a + b), ee = 0.5 * (b - a);
        if (!(ee > 0.0)) break;
        double *y0 = x, *y1 = t1, *y2 = t2;
        HIP_TRY(hd::launch_eig_cheb(N, rowptr, col, val, m, y0, nullptr, y1, 1.0 / ee, -cc / ee, 0.0, s));
        for (int d = 2; d <= opts->degree; ++d) {
            double *yout = d == 2 ? y2 : y0 == x ? sx : y0;  // keep the result out of the buffers in use
            HIP_TRY(hd::launch_eig_cheb(N, rowptr, col, val, m, y1, y0, yout, 2.0 / ee, -2.0 * cc / ee, -1.0, s));
            y0 = y1;
            y1 = yout;
        }
        // the filtered block is y1; make it X (the other buffers are free)
        if (y1 != x) {
            if (y1 == sx) std::swap(x, sx);
            else if (y1 == t1) std::swap(x, t1);
            else std::swap(x, t2);
        }
        // x holds the filtered block; t1 is free for the out-of-place
        // rotations (orth exchanges the two pointers)
        e = orth(x, t1);
        if (e != HD_OK) return e;
    }
    if (lambda_out) std::copy(w.begin(), w.begin() + r, lambda_out);
    if (resid_out) std::copy(res.begin(), res.begin() + r, resid_out);
    // U1 = the r leading columns, to the host, then loaded in the requested form
    DevBuf Uf;
    HIP_TRY(Uf.ensure((size_t)N * r * sizeof(float)));
    HIP_TRY(hd::launch_eig_extract(N, m, r, x, Uf.as<float>(), s));
    std::vector<float> hU((size_t)N * r);
    HIP_TRY(hipMemcpy(hU.data(), Uf.p, hU.size() * sizeof(float), hipMemcpyDeviceToHost));
    if (U_out) std::copy(hU.begin(), hU.end(), U_out);
    for (DevBuf *bf : {&X, &SX, &T1, &T2, &Uf}) bf->release();
    // the eigensolver's rounding can put lambda_1 a hair above 1
    std::vector<double> lam(w.begin(), w.begin() + r);
    for (double &l : lam) l = std::max(-1.0, std::min(1.0, l));
    c->eig_outer = outer + 1;
    return hd_load_eigs(c, r, hU.data(), lam.data(), dtype);
}

}  // extern "C"

extern "C" int32_t hd_eig_steps(const hd_ctx *c) { return c ? c->eig_outer : 0; }
