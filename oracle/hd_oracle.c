/*
 * FP64 oracle for hybrid spectral-temporal diffusion (Iscen, Avrithis, Tolias,
 * Furon, Chum: "Hybrid Diffusion: Spectral-Temporal Graph Filtering for
 * Manifold Ranking").
 *
 * TEST INFRASTRUCTURE ONLY. This file is the plain, slow, single-threaded
 * reference that the GPU library is checked against. It shares no code,
 * header, table or helper with the HIP path, and the product path never
 * links or calls it. Only the test suite, the smoke check and the CPU
 * baseline leg of the benchmark load it.
 *
 * Every quantity is double precision. Inputs stored by the caller in single
 * precision (graph values, descriptors, eigenvectors) are widened to double
 * by the Python wrapper before they reach these functions.
 *
 * Functions, and the passage each one follows:
 *   hdo_normalize    Section 3 (problem formulation): W -> D^-1/2 W D^-1/2
 *   hdo_csr_matvec   Section 3: product with the sparse normalised adjacency
 *   hdo_observation  Section 3 and Section 6.1 (implementation details):
 *                    sparse observation vector y from the query's nearest
 *                    neighbours, entries (v^T z)_+^3
 *   hdo_spectral     Section 4.2, eq. (h-spectral): x^s = U1 g(L1) U1^T y
 *   hdo_cg           Section 4.2, eqs. (h-temporal) and (box); Section 5:
 *                    conjugate gradient from x0 = 0 on the deflated system
 *   hdo_rank         Section 3: ranking by decreasing x
 *
 * Readings of points the paper leaves open (ties, stopping rule, breakdown)
 * are stated beside the code that takes them.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* Per-column outcome of the iterative solve. */
enum { HDO_CONVERGED = 0, HDO_MAXITER = 1, HDO_ZERO_RHS = 2, HDO_BREAKDOWN = 3 };

/*
 * Section 3: D = diag(W 1), and the normalised adjacency is
 * D^-1/2 W D^-1/2. A node with zero degree has no edges, so its row and
 * column are zero; it is given a zero scale rather than a division by zero.
 * The two scales are multiplied first so that S is exactly symmetric when W
 * is.
 * s_out has the same sparsity pattern as w.
 */
int hdo_normalize(int64_t n, const int64_t *rowptr, const int32_t *col,
                  const double *w, double *s_out)
{
    double *dinv = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    if (!dinv) return -1;
    for (int64_t i = 0; i < n; ++i) {
        double deg = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) deg += w[e];
        dinv[i] = deg > 0.0 ? 1.0 / sqrt(deg) : 0.0;
    }
    for (int64_t i = 0; i < n; ++i)
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e)
            s_out[e] = w[e] * (dinv[i] * dinv[col[e]]);   /* symmetric in i, j */
    free(dinv);
    return 0;
}

/* out = S z for CSR S (Section 3: S is sparse, so this costs O(nnz)). */
void hdo_csr_matvec(int64_t n, const int64_t *rowptr, const int32_t *col,
                    const double *val, const double *z, double *out)
{
    for (int64_t i = 0; i < n; ++i) {
        double acc = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) acc += val[e] * z[col[e]];
        out[i] = acc;
    }
}

/* True when (s1, j1) ranks ahead of (s2, j2): larger score first, and on
 * equal scores the lower item id first. */
static int ahead(double s1, int64_t j1, double s2, int64_t j2)
{
    return s1 > s2 || (s1 == s2 && j1 < j2);
}

/*
 * Sections 3 and 6.1: the observation vector y of one query. Its non-zero
 * entries sit at the k database items most similar to the query, and each
 * holds the similarity (v^T z)_+^3 = max(0, v^T z)^3. Descriptors are
 * unit-norm, so v^T z is the cosine. Equal similarities go to the lower id.
 *   V: n x d row-major database descriptors; q: d query descriptor.
 *   ids_out / val_out: k entries, best first.
 */
int hdo_observation(int64_t n, int64_t d, const double *V, const double *q,
                    int32_t k, int32_t *ids_out, double *val_out)
{
    if (k < 0 || k > n) return -1;
    double *best_s = (double *)malloc(sizeof(double) * (size_t)(k > 0 ? k : 1));
    int64_t *best_j = (int64_t *)malloc(sizeof(int64_t) * (size_t)(k > 0 ? k : 1));
    if (!best_s || !best_j) { free(best_s); free(best_j); return -1; }
    int32_t have = 0;
    for (int64_t j = 0; j < n; ++j) {
        double s = 0.0;
        const double *v = V + j * d;
        for (int64_t t = 0; t < d; ++t) s += q[t] * v[t];
        /* keep the k best seen so far, sorted best first (insertion) */
        if (have < k) {
            int32_t pos = have++;
            while (pos > 0 && ahead(s, j, best_s[pos - 1], best_j[pos - 1])) {
                best_s[pos] = best_s[pos - 1];
                best_j[pos] = best_j[pos - 1];
                --pos;
            }
            best_s[pos] = s;
            best_j[pos] = j;
        } else if (k > 0 && ahead(s, j, best_s[k - 1], best_j[k - 1])) {
            int32_t pos = k - 1;
            while (pos > 0 && ahead(s, j, best_s[pos - 1], best_j[pos - 1])) {
                best_s[pos] = best_s[pos - 1];
                best_j[pos] = best_j[pos - 1];
                --pos;
            }
            best_s[pos] = s;
            best_j[pos] = j;
        }
    }
    for (int32_t t = 0; t < k; ++t) {
        double c = best_s[t] > 0.0 ? best_s[t] : 0.0;
        ids_out[t] = (int32_t)best_j[t];
        val_out[t] = c * c * c;
    }
    free(best_s);
    free(best_j);
    return 0;
}

/* Transfer function of Section 3, eq. (transfer), on one eigenvalue:
 * h(x) = (1 - alpha) / (1 - alpha x). */
static double h_alpha(double alpha, double x) { return (1.0 - alpha) / (1.0 - alpha * x); }

/* Theorem of Section 4.1, eq. (aux): g(x) = h(x) - h(0). */
static double g_alpha(double alpha, double x) { return h_alpha(alpha, x) - h_alpha(alpha, 0.0); }

/*
 * Section 4.2, eq. (h-spectral): x^s = U1 g(L1) U1^T y, evaluated right to
 * left. y is sparse (k entries). U is n x r row-major (item-major), lam has
 * the r eigenvalues that go with U's columns.
 */
int hdo_spectral(int64_t n, int32_t r, const double *U, const double *lam,
                 double alpha, int32_t k, const int32_t *y_ids, const double *y_val,
                 double *xs_out)
{
    double *c = (double *)calloc((size_t)(r > 0 ? r : 1), sizeof(double));
    if (!c) return -1;
    for (int32_t t = 0; t < k; ++t) {               /* c = U1^T y */
        const double *u = U + (int64_t)y_ids[t] * r;
        for (int32_t j = 0; j < r; ++j) c[j] += u[j] * y_val[t];
    }
    for (int32_t j = 0; j < r; ++j) c[j] *= g_alpha(alpha, lam[j]);   /* g(L1) c */
    for (int64_t i = 0; i < n; ++i) {                /* U1 (g(L1) c) */
        double acc = 0.0;
        const double *u = U + i * r;
        for (int32_t j = 0; j < r; ++j) acc += u[j] * c[j];
        xs_out[i] = acc;
    }
    free(c);
    return 0;
}

/*
 * Section 4.2, eq. (box): the black-box product of the deflated regularised
 * Laplacian,
 *     z -> (z - alpha (S z - U1 L1 U1^T z)) / (1 - alpha),
 * with U1 L1 U1^T z taken right to left (U1^T z, then L1, then U1).
 * work must hold r doubles.
 */
static void deflated_apply(int64_t n, const int64_t *rowptr, const int32_t *col,
                           const double *val, int32_t r, const double *U,
                           const double *lam, double alpha, const double *z,
                           double *out, double *work)
{
    for (int32_t j = 0; j < r; ++j) work[j] = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        const double *u = U + i * r;
        for (int32_t j = 0; j < r; ++j) work[j] += u[j] * z[i];
    }
    for (int32_t j = 0; j < r; ++j) work[j] *= lam[j];
    for (int64_t i = 0; i < n; ++i) {
        double sz = 0.0;
        for (int64_t e = rowptr[i]; e < rowptr[i + 1]; ++e) sz += val[e] * z[col[e]];
        double uz = 0.0;
        const double *u = U + i * r;
        for (int32_t j = 0; j < r; ++j) uz += u[j] * work[j];
        out[i] = (z[i] - alpha * (sz - uz)) / (1.0 - alpha);
    }
}

static double dot(int64_t n, const double *a, const double *b)
{
    double s = 0.0;
    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];
    return s;
}

/*
 * Section 4.2, eq. (h-temporal), solved as Section 5 describes: conjugate
 * gradient (Hestenes-Stiefel) on L(S - U1 L1 U1^T) x = y from x0 = 0, the
 * matrix reached only through the product of eq. (box). With r = 0 this is
 * plain temporal filtering, eq. (temporal).
 *
 * Readings taken where the paper is silent:
 *  - the iteration count is the number of operator products;
 *  - a column stops when sqrt(rho_i / rho_0) <= tol, rho = r^T r of the
 *    recurrence residual, tested right after the x and r updates; tol <= 0
 *    runs exactly max_iter products unless the residual reaches zero;
 *  - y = 0 gives x = 0 with status ZERO_RHS and no iteration;
 *  - gamma = p^T A p that is not positive and finite stops the column with
 *    status BREAKDOWN, keeping the last x.
 * Outputs: x (n), *iters, *relres = sqrt(rho/rho_0) at exit, *status.
 */
int hdo_cg(int64_t n, const int64_t *rowptr, const int32_t *col, const double *val,
           int32_t r, const double *U, const double *lam, double alpha,
           const double *y, int32_t max_iter, double tol,
           double *x, int32_t *iters, double *relres, int32_t *status)
{
    size_t nn = (size_t)(n > 0 ? n : 1);
    double *res = (double *)malloc(sizeof(double) * nn);
    double *p = (double *)malloc(sizeof(double) * nn);
    double *q = (double *)malloc(sizeof(double) * nn);
    double *work = (double *)malloc(sizeof(double) * (size_t)(r > 0 ? r : 1));
    if (!res || !p || !q || !work) { free(res); free(p); free(q); free(work); return -1; }

    for (int64_t i = 0; i < n; ++i) { x[i] = 0.0; res[i] = y[i]; p[i] = y[i]; }
    double rho0 = dot(n, y, y);
    double rho = rho0;
    *iters = 0;
    if (!(rho0 > 0.0)) {
        *relres = 0.0;
        *status = rho0 == 0.0 ? HDO_ZERO_RHS : HDO_BREAKDOWN;
        free(res); free(p); free(q); free(work);
        return 0;
    }
    *status = HDO_MAXITER;
    for (int32_t it = 1; it <= max_iter; ++it) {
        deflated_apply(n, rowptr, col, val, r, U, lam, alpha, p, q, work);
        double gamma = dot(n, p, q);
        if (!(gamma > 0.0) || !isfinite(gamma)) { *status = HDO_BREAKDOWN; break; }
        double a = rho / gamma;
        for (int64_t i = 0; i < n; ++i) { x[i] += a * p[i]; res[i] -= a * q[i]; }
        double rho_new = dot(n, res, res);
        *iters = it;
        if (sqrt(rho_new / rho0) <= tol) { rho = rho_new; *status = HDO_CONVERGED; break; }
        double beta = rho_new / rho;
        for (int64_t i = 0; i < n; ++i) p[i] = res[i] + beta * p[i];
        rho = rho_new;
    }
    *relres = sqrt(rho / rho0);
    free(res); free(p); free(q); free(work);
    return 0;
}

/* Section 3: items are ranked by decreasing x; equal values go to the lower
 * id. Each sort element carries its score and id, so the comparison needs no
 * shared state and calls may run on several threads at once. */
typedef struct {
    double x;
    int64_t id;
} rank_item;

static int rank_cmp(const void *a, const void *b)
{
    const rank_item *u = (const rank_item *)a, *v = (const rank_item *)b;
    if (u->x > v->x) return -1;
    if (u->x < v->x) return 1;
    return (u->id > v->id) - (u->id < v->id);
}

/* Top-K of the ranking: ids_out / score_out get the K best items in order. */
int hdo_rank(int64_t n, const double *x, int32_t K, int32_t *ids_out, double *score_out)
{
    if (K < 0 || K > n) return -1;
    rank_item *it = (rank_item *)malloc(sizeof(rank_item) * (size_t)(n > 0 ? n : 1));
    if (!it) return -1;
    for (int64_t i = 0; i < n; ++i) {
        it[i].x = x[i];
        it[i].id = i;
    }
    qsort(it, (size_t)n, sizeof(rank_item), rank_cmp);
    for (int32_t t = 0; t < K; ++t) { ids_out[t] = (int32_t)it[t].id; score_out[t] = it[t].x; }
    free(it);
    return 0;
}
