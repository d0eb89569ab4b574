// (r, i) planner: how many eigenpairs to deflate and how many CG iterations
// to run, from the spectrum and a per-iteration cost.
//
// Section 5 bounds the A-norm error of CG on the deflated system by
//   ||e_i||_A <= 2 ((sqrt(k) - 1) / (sqrt(k) + 1))^i ||e_0||_A      (eq. (bound))
// with k = (1 - a lambda_n) / (1 - a lambda_{r+1}) for r deflated pairs
// (eq. (cond-r)). When a few of the next eigenvalues stand apart from the
// rest (lambda_1 = 1 above a gap is the typical case), the bound is refined
// the classical way: CG spends one iteration on each of m outlying
// eigenvalues of A at the small end (lambda_{r+1} .. lambda_{r+m} of the
// graph) and then converges at the rate of the remaining interval; the
// polynomial that removes them can grow the error on that interval by
//   F_m = prod_j (A_max / A_j - 1),  A_j = (1 - a lambda_j) / (1 - a),
// so i(r) = min over m of  m + ceil(ln(2 F_m / eps) / ln((sqrt(k_m) + 1) / (sqrt(k_m) - 1))).
// The predicted time of a candidate is fixed_ms + i(r) iter_ms, with the costs
// measured by the caller.
#include <cmath>
#include <cstdint>

#include "hd_internal.h"

namespace {

// iterations guaranteed by the bound for deflated rank r (lambda: the nlam
// leading eigenvalues of S, descending; lambda_{r+1} beyond them is taken
// as lambda_nlam, an upper value)
int32_t bound_iters(int32_t nlam, const double *lambda, double lmin, double alpha, double eps, int32_t r,
                    int32_t max_out) {
    const double amax = 1.0 - alpha * lmin;  // (1 - alpha) A_max
    auto lam_at = [&](int32_t j) -> double {  // lambda_{j+1}, 0-based j
        const double l = j < nlam ? lambda[j] : lambda[nlam - 1];
        return l > 0.0 ? l : 0.0;             // deflated directions sit at 0
    };
    double best = 1e300;
    double logF = 0.0;
    for (int32_t m = 0; m <= max_out && r + m <= nlam; ++m) {
        if (m > 0) {
            const double aj = 1.0 - alpha * lam_at(r + m - 1);
            const double f = amax / aj - 1.0;
            if (f > 1.0) logF += std::log(f);
        }
        const double k = amax / (1.0 - alpha * lam_at(r + m));
        double it;
        if (k <= 1.0 + 1e-12) {
            it = m + 1;
        } else {
            const double sk = std::sqrt(k);
            const double rate = std::log((sk + 1.0) / (sk - 1.0));
            it = m + std::ceil((std::log(2.0 / eps) + logF) / rate);
        }
        if (it < best) best = it;
    }
    return best > 1e9 ? INT32_MAX : (int32_t)best;
}

}  // namespace

extern "C" {

int hd_rank_plan(int32_t nlam, const double *lambda, double lambda_min, double alpha, double eps,
                 int32_t ncand, const int32_t *cand_r, const double *fixed_ms, const double *iter_ms,
                 int32_t *iters_out, double *pred_ms_out, int32_t *best) {
    g_err.clear();
    if (nlam < 1 || !lambda) return fail(HD_EINVAL, "hd_rank_plan: need at least one eigenvalue");
    if (!(alpha > 0.0 && alpha < 1.0)) return fail(HD_EINVAL, "hd_rank_plan: alpha=%g not in (0, 1)", alpha);
    if (!(eps > 0.0 && eps < 1.0)) return fail(HD_EINVAL, "hd_rank_plan: eps=%g not in (0, 1)", eps);
    if (!(lambda_min >= -1.0 - 1e-6 && lambda_min <= lambda[nlam - 1]))
        return fail(HD_EINVAL, "hd_rank_plan: lambda_min=%g not in [-1, lambda_nlam]", lambda_min);
    for (int32_t j = 0; j < nlam; ++j) {
        if (!(std::fabs(lambda[j]) <= 1.0 + 1e-6)) return fail(HD_EINVAL, "hd_rank_plan: lambda[%d] outside [-1, 1]", j);
        if (j > 0 && lambda[j] > lambda[j - 1]) return fail(HD_EINVAL, "hd_rank_plan: lambda not descending");
    }
    if (ncand < 1 || !cand_r || !iters_out) return fail(HD_EINVAL, "hd_rank_plan: no candidates");
    double best_ms = 1e300;
    if (best) *best = -1;
    for (int32_t c = 0; c < ncand; ++c) {
        const int32_t r = cand_r[c];
        if (r < 0 || r > nlam) return fail(HD_EINVAL, "hd_rank_plan: candidate r=%d not in [0, %d]", r, nlam);
        iters_out[c] = bound_iters(nlam, lambda, lambda_min, alpha, eps, r, 64);
        if (fixed_ms && iter_ms) {
            const double ms = fixed_ms[c] + iters_out[c] * iter_ms[c];
            if (pred_ms_out) pred_ms_out[c] = ms;
            if (ms < best_ms) {
                best_ms = ms;
                if (best) *best = c;
            }
        }
    }
    return HD_OK;
}

}  // extern "C"
