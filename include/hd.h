/*
 * hd.h - C ABI of the MI355X (gfx950) query path of hybrid spectral-temporal
 * diffusion (Iscen, Avrithis, Tolias, Furon, Chum, "Hybrid Diffusion:
 * Spectral-Temporal Graph Filtering for Manifold Ranking").
 *
 * The library answers batches of queries against a resident database:
 *   1. the observation vector y of each query: its k_y most similar database
 *      items, with entries max(0, cos)^3 (Section 3; Section 6.1);
 *   2. the spectral term x^s = U1 g(L1) U1^T y (Section 4.2, eq. (h-spectral));
 *   3. the temporal term x^t, conjugate gradient from x0 = 0 on
 *      L(S - U1 L1 U1^T) x^t = y through the product of eq. (box)
 *      (Section 4.2, eq. (h-temporal); Section 5);
 *   4. the ranking of x = x^s + x^t by decreasing value (Section 3,
 *      eq. (hybrid)).
 *
 * Conventions for every entry point:
 *   - The return value is an hd_status: HD_OK (0) on success, a negative
 *     code on failure. No entry point aborts or throws; hd_last_error()
 *     returns a message for the last failure on the calling thread.
 *   - "host" pointers are ordinary CPU memory; "device" pointers are GPU
 *     memory on the context's device (for instance a torch tensor's
 *     data_ptr()). Each argument says which it takes.
 *   - Loaders copy their inputs: the caller may free them on return. The
 *     library owns every device buffer it allocates and frees them in
 *     hd_destroy(). It never frees caller memory.
 *   - A context is used by one host thread at a time.
 *   - Queries run on the HIP stream passed in (NULL = the default stream).
 */
#ifndef HD_H
#define HD_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct hd_ctx hd_ctx;

typedef enum {
    HD_OK = 0,
    HD_EINVAL = -1,   /* an argument or an input array is invalid          */
    HD_ENOMEM = -2,   /* a device or host allocation failed                */
    HD_EDEVICE = -3,  /* a HIP runtime call or kernel launch failed        */
    HD_ESTATE = -4    /* call out of order (e.g. query before load_graph)  */
} hd_status;

/* Outcome of one query column of the conjugate-gradient solve. */
typedef enum {
    HD_COL_CONVERGED = 0,  /* relative residual reached the tolerance        */
    HD_COL_MAXITER = 1,    /* stopped at the iteration cap                   */
    HD_COL_ZERO_RHS = 2,   /* y = 0: x = 0, no iteration                     */
    HD_COL_BREAKDOWN = 3   /* p^T A p not positive and finite: stopped, last x kept */
} hd_col_status;

/* Storage precision of the eigenvectors U1 and of the database descriptors. */
typedef enum {
    HD_F32 = 0,
    HD_BF16 = 1,          /* bfloat16, rounded to nearest even from the fp32 input */
    HD_FP8_E4M3 = 2,      /* OCP FP8 E4M3 codes (bias 7, max 448, no infinities)
                             with one fp32 scale per column (U1) or per row (V):
                             value = scale * code value */
    HD_BF16X2 = 3,        /* U1 only: two bfloat16 terms hi + lo, hi = RNE(u),
                             lo = RNE(u - hi) (about 16 significant bits) */
    HD_SPARSE_F32 = 4     /* U1 only, set by hd_load_eigs_sparse: sparsified
                             fp32 U1 (SHybrid) */
} hd_dtype;

/* hd_load_graph flags. */
#define HD_GRAPH_NORMALIZE 1u   /* val holds W; store D^-1/2 W D^-1/2 (Section 3) */
#define HD_GRAPH_CHECK_SYMMETRY 2u  /* verify W = W^T (costs one pass over the edges) */

/*
 * Create a context on HIP device `device` (index as seen by this process).
 * *out receives the context. Errors: HD_EINVAL (bad device or NULL out),
 * HD_EDEVICE.
 */
int hd_create(int device, hd_ctx **out);

/* Release every device buffer of the context and the context itself.
 * NULL is accepted. Waits for work queued by the context to finish. */
void hd_destroy(hd_ctx *ctx);

/* Message of the last failed call on this thread ("" if none). The string
 * stays valid until the next call on this thread. */
const char *hd_last_error(void);

/*
 * Load the graph (Section 3): n items, a sparse symmetric non-negative
 * zero-diagonal matrix in CSR form with int64 row pointers (host, n+1),
 * int32 column ids (host, nnz) sorted within each row, and fp32 values
 * (host, nnz). Without HD_GRAPH_NORMALIZE the values are taken as the
 * normalised S = D^-1/2 W D^-1/2; with it they are W and the library
 * normalises (in double precision, exactly symmetric; an item of zero
 * degree gets a zero row). Replaces any previous graph and drops any loaded
 * eigenpairs and descriptors of another size.
 * Errors (HD_EINVAL): n <= 0 or n >= 2^31, rowptr not starting at 0,
 * decreasing or not ending at nnz, a column out of range, unsorted or
 * repeated within its row, a diagonal entry, a negative or non-finite
 * value, or (with HD_GRAPH_CHECK_SYMMETRY) an asymmetric matrix.
 */
int hd_load_graph(hd_ctx *ctx, int64_t n, int64_t nnz, const int64_t *rowptr,
                  const int32_t *col, const float *val, uint32_t flags);

/*
 * Load r eigenpairs of S (Section 4.1: U1 is n x r with orthonormal
 * columns, L1 = diag(lambda)), the input of eqs. (h-spectral) and (box).
 * U (host, fp32, n x r row-major: row i holds item i's r components),
 * lambda (host, double, r values, each in [-1, 1] up to 1e-6 of rounding). `dtype` selects the
 * storage precision on the device: HD_F32, or HD_BF16 (U rounded to
 * nearest-even bfloat16 and kept twice, item-major and component-major,
 * each in the matrix cores' 16 x 32 operand-tile order; the
 * products multiply it with the fp32 operand split into two bfloat16 parts
 * and accumulate in fp32), or HD_BF16X2 (U kept as two bfloat16 terms in
 * both layouts, products over three bfloat16 terms, accuracy close to fp32
 * at twice the bytes of HD_BF16), or HD_FP8_E4M3 (each column k quantized
 * as by hd_quantize_fp8_e4m3 with one scale per column and kept as one-byte
 * codes in the same two layouts; the products convert the codes to bfloat16
 * in registers, which is exact, and apply the scales to the small
 * coefficient matrices). r = 0 unloads. Queries may use any prefix of the
 * loaded columns (hd_query_opts.rank_r).
 * Every argument is checked before the context changes: a rejected call
 * leaves the loaded eigenpairs as they were. A failure after the checks (an
 * allocation or a copy) leaves no eigenpairs loaded.
 * Errors: HD_ESTATE (no graph), HD_EINVAL (r < 0, r > n, lambda outside
 * [-1, 1] or non-finite, non-finite U, unknown dtype).
 */
int hd_load_eigs(hd_ctx *ctx, int32_t r, const float *U, const double *lambda,
                 int32_t dtype);

/*
 * Load r eigenpairs with U1 already in the FP8 form (the storage precision of
 * the precision form; Section 4.1 defines U1): codes (host, n x r row-major
 * OCP FP8 E4M3 bytes, so U1[i][k] = col_scale[k] * value(codes[i r + k])),
 * col_scale (host, r fp32 values > 0), lambda (host, r doubles in [-1, 1]).
 * Same device layout and queries as hd_load_eigs with HD_FP8_E4M3, and the
 * same rule on rejected calls.
 * Errors: HD_ESTATE (no graph), HD_EINVAL (r not in [1, n], NULL array, a NaN
 * code 0x7F / 0xFF, a scale not positive and finite, lambda out of range).
 */
int hd_load_eigs_fp8(hd_ctx *ctx, int32_t r, const uint8_t *codes, const float *col_scale,
                     const double *lambda);

/*
 * The FP8 quantizer of the precision form (host only, no device work): for a
 * rows x cols row-major fp32 matrix A (host), one scale per column
 * (per_column != 0, scales[cols]) or per row (per_column = 0, scales[rows]),
 * scale = max |a| / 448 over the line (1 for an all-zero line, division in
 * fp32), and codes[i cols + k] (host) = a / scale rounded to the nearest OCP
 * FP8 E4M3 value, ties to even, magnitudes at or above 448 saturating to 448.
 * Errors: HD_EINVAL (negative size, NULL array, non-finite input).
 */
int hd_quantize_fp8_e4m3(int64_t rows, int32_t cols, const float *A, int32_t per_column,
                         uint8_t *codes, float *scales);

/*
 * Launch parameters of the hot kernels: the search space of hd_autotune.
 * Value 0 selects the built-in default; a value that does not fit the
 * solver width of a call (1, 2 or 4, dividing the width in 64-column units)
 * falls back to the default for that call.
 */
typedef enum {
    HD_TUNE_SPMM_CPL = 0,  /* sparse product: query columns per lane (1, 2, 4) */
    HD_TUNE_UTP_NT = 1,    /* U1^T P, bfloat16 forms: 16-column tiles per wave */
    HD_TUNE_UC_NT = 2,     /* U1 C and the final combine, bfloat16 forms: same */
    HD_TUNE_SPMM_BANDS = 3, /* sparse product: source bands (1, 2, 4, 8): each
                              row's neighbours split by neighbour id into that
                              many runs, one launch per run, so that the rows
                              of P gathered at one time fit the device's
                              memory-side cache; bit-identical results */
    HD_TUNE_TOPK_ONEPASS = 4, /* top-k of the similarities (bfloat16 or fp8
                              descriptors) and the final top-K (plain CG or
                              the matrix-core U1 forms, no x output) for
                              n >= 65536 items: 0 or 2 one pass (a sampled
                              threshold per row, candidates taken from the
                              scores as they are produced, no score matrix
                              written unless a row needs the exact
                              fallback), 1 two passes (the score matrix,
                              then the selection); identical results */
    HD_TUNE_NKEYS = 5
} hd_tune_key;

/* Set / read one launch parameter. Errors: HD_EINVAL (key, value not in
 * {0, 1, 2, 4}, {0, 1, 2, 4, 8} for HD_TUNE_SPMM_BANDS, {0, 1, 2} for
 * HD_TUNE_TOPK_ONEPASS; NULL). */
int hd_set_tuning(hd_ctx *ctx, int32_t key, int32_t value);
int hd_get_tuning(const hd_ctx *ctx, int32_t key, int32_t *value);

/*
 * Autotuner (batching form): for batches of `batch` queries, time every
 * valid value of each launch parameter on the loaded graph and eigenvectors
 * (one warm-up and `reps` timed launches each, on device scratch vectors of
 * the solver width, on the null stream) and keep the fastest in the
 * context; the built-in default is kept unless a candidate beats it by more
 * than 2%. The sparse product's two parameters (columns per lane, source
 * bands) are tuned together over every pair; more than one band is kept
 * only when 5% faster than the best single pass. times_ms (host, may be NULL)
 * receives HD_TUNE_NKEYS x 4 mean launch times in ms for the values 1, 2,
 * 4, 8 (-1 where a value does not fit or the kernel is not used: no
 * eigenvectors, or fp32 storage); for the two sparse-product keys, the time
 * of that value with the other key at its chosen value. HD_TUNE_TOPK_ONEPASS
 * is not searched (its times are -1, its value unchanged).
 * Synchronous. Errors: HD_ESTATE (no graph), HD_EINVAL (batch not in
 * [1, 1024], reps not in [1, 1000]).
 */
int hd_autotune(hd_ctx *ctx, int32_t batch, int32_t reps, double *times_ms);

/*
 * Persistent CG (batching form): with mode 1 (batches of at most 16 queries)
 * or 2 (at most 64), hd_query_batch, hd_plan_create and hd_plan_run run
 * every CG iteration of an eligible batch in one kernel (Section 5: CG; the
 * operator of Section 4.2, eq. (box)): solver vectors W columns wide (the
 * batch size rounded up to a power of two, instead of at least 64), blocks
 * co-resident and separated by grid barriers, scalars reduced in a fixed
 * order by the last block to reach each barrier. Eligible: plain CG (rank 0)
 * or fp32 U1 with at most 1024 components in use and at most 16 queries, no
 * polynomial filter. Other batches take the multi-kernel path. Mode 0 (the
 * default) turns it off. Results agree with the multi-kernel path to fp32
 * rounding (its partial sums are grouped differently); each column is
 * still independent of the others. spin_limit (> 0; 0 = the default, 2^24):
 * the bound on each barrier wait, in polling rounds; a wait past it ends
 * the kernel early and the call returns HD_EDEVICE.
 * Errors: HD_EINVAL (NULL context, mode not in {0, 1, 2}, spin_limit < 0).
 */
int hd_set_persistent(hd_ctx *ctx, int32_t mode, int64_t spin_limit);

/*
 * (r, i) planner (Section 5, eqs. (bound) and (cond-r)): for each candidate
 * number of deflated eigenpairs cand_r[c] (0 <= r <= nlam), the number of CG
 * iterations that the error bound guarantees to bring the relative A-norm
 * error below eps, refined for up to 64 outlying eigenvalues above the rest;
 * with per-candidate costs (fixed_ms: y, spectral term, combine and ranking;
 * iter_ms: one CG iteration; both may be NULL) also the predicted time and
 * the fastest candidate. lambda (host, nlam values): the leading eigenvalues
 * of S, descending (the loaded Lambda1); lambda_min: a lower value for the
 * smallest eigenvalue of S (-1 is always valid); eigenvalues past nlam are
 * taken as lambda[nlam-1]. Host only; no device work.
 * Outputs (host): iters_out[ncand], pred_ms_out[ncand] (may be NULL), *best
 * (index of the fastest candidate, -1 without costs; may be NULL).
 * Errors: HD_EINVAL (arguments).
 */
int hd_rank_plan(int32_t nlam, const double *lambda, double lambda_min, double alpha, double eps,
                 int32_t ncand, const int32_t *cand_r, const double *fixed_ms, const double *iter_ms,
                 int32_t *iters_out, double *pred_ms_out, int32_t *best);

/*
 * On-device top-r eigensolver (the off-line input of Section 4.1): computes
 * the r algebraically largest eigenpairs of the loaded S by Chebyshev-filtered
 * subspace iteration in double precision on a block of r + guard vectors
 * (rounded up to a multiple of 64), then loads them as hd_load_eigs does with
 * `dtype` (HD_F32, HD_BF16, HD_BF16X2). Stops when the r leading residual
 * norms ||S u_j - lambda_j u_j|| are <= tol, after max_outer Rayleigh-Ritz
 * steps, or past time_budget_s (0: no limit). lambda_min: a lower value for
 * the smallest eigenvalue of S (-1 is always valid). Device memory: about
 * 4 N (r + guard) doubles while it runs. Outputs (host, may be NULL):
 * lambda_out[r] (descending), resid_out[r], U_out[n x r] (fp32, item-major).
 * Errors: HD_ESTATE (no graph), HD_EINVAL (options), HD_ENOMEM, HD_EDEVICE
 * (a library call or factorisation failed).
 */
typedef struct {
    int32_t guard;         /* extra block vectors beyond r (>= 1)            */
    int32_t degree;        /* Chebyshev filter degree per step, [1, 64]      */
    int32_t max_outer;     /* Rayleigh-Ritz steps at most                    */
    double tol;            /* residual norm target                           */
    double time_budget_s;  /* wall-clock limit, 0 = none                     */
    uint64_t seed;         /* start block (counter-based normal draws)       */
    double lambda_min;     /* lower end of the damped interval               */
} hd_eig_opts;
int hd_compute_eigs(hd_ctx *ctx, int32_t r, int32_t dtype, const hd_eig_opts *opts, double *lambda_out,
                    double *resid_out, float *U_out);
/* Rayleigh-Ritz steps taken by the last successful hd_compute_eigs on ctx
 * (0 before any, and for NULL). */
int32_t hd_eig_steps(const hd_ctx *ctx);

/*
 * SHybrid (Section 6.2): load a sparsified U1 (most entries set to zero,
 * not renormalised) and its eigenvalues; the hybrid method then runs with
 * sparse eigenvector products (one wave per item or component, gathering
 * rows of the small dense operand). U~ is given by item in CSR form (host):
 * rowptr[n+1] (int64, from 0, non-decreasing, ending at nnz), col[nnz]
 * (component ids in [0, r), strictly increasing within a row), val[nnz]
 * (fp32, finite); lambda as for hd_load_eigs. The library keeps the CSR and
 * builds the by-component (CSC) copy. Replaces any loaded eigenpairs; queries
 * may use a prefix rank_r as with dense U1. The continuous-batching server
 * does not take sparse U1 (HD_ESTATE from hd_serve_open).
 * Errors: HD_ESTATE (no graph), HD_EINVAL (r, arrays, lambda).
 */
int hd_load_eigs_sparse(hd_ctx *ctx, int32_t r, int64_t nnz, const int64_t *rowptr, const int32_t *col,
                        const float *val, const double *lambda);

/*
 * Load the database descriptors used to build y from query descriptors
 * (Section 3: nearest neighbours of the query in the dataset). V (host,
 * fp32, n x d row-major, unit-norm rows so that the dot product is the
 * cosine). `dtype` selects the device storage: HD_F32, or HD_BF16 (rounded to
 * nearest even and kept in the matrix cores' 16 x 32 operand-tile order;
 * the query descriptors stay fp32 and are split into two bfloat16 parts for
 * the product), or HD_FP8_E4M3 (each row quantized as by
 * hd_quantize_fp8_e4m3 with one scale per row, codes in the same operand
 * order, converted to bfloat16 in registers; the scale multiplies the row's
 * similarities). HD_BF16X2 is not accepted here. The host arrays are
 * converted on the host and may be freed on return. A rejected call leaves
 * the loaded descriptors as they were; a failure after the checks leaves
 * none loaded.
 * Errors: HD_ESTATE (no graph), HD_EINVAL (d <= 0, non-finite V, dtype).
 */
int hd_load_descriptors(hd_ctx *ctx, int32_t d, const float *V, int32_t dtype);

/*
 * Load descriptors already in the FP8 form: codes (host, n x d row-major OCP
 * FP8 E4M3 bytes, V[i][t] = row_scale[i] * value(codes[i d + t])), row_scale
 * (host, n fp32 values > 0). Same use as hd_load_descriptors with
 * HD_FP8_E4M3 and the same rule on rejected calls.
 * Errors: HD_ESTATE (no graph), HD_EINVAL (d <= 0, NULL array, a NaN code, a
 * scale not positive and finite).
 */
int hd_load_descriptors_fp8(hd_ctx *ctx, int32_t d, const uint8_t *codes, const float *row_scale);

/* Options of one query batch. */
typedef struct {
    double alpha;      /* Section 3: alpha in [0, 1); the paper uses 0.99      */
    int32_t max_iter;  /* CG iteration cap (number of operator products), >= 0 */
    double tol;        /* stop a column when sqrt(r^T r / y^T y) <= tol (after
                          the x and r updates); tol <= 0 runs max_iter products.
                          tol < 0 (hd_query_batch and plans, multi-kernel
                          path): as 0, except that the last product updates
                          x alone and forms no residual (nothing else reads
                          it), so relres reports the residual before it */
    int32_t rank_r;    /* use the first rank_r loaded eigenpairs (0 = plain CG,
                          the temporal filtering of eq. (temporal)); -1 = all  */
    int32_t k_y;       /* non-zeros of y per query, 1..min(n, 1024)             */
    int32_t top_k;     /* K of the ranking, 0 (none) .. min(n, 1024)           */
} hd_query_opts;

/*
 * Answer B queries, 1 <= B <= 1024 (the whole path above, steps 1-4).
 * Query input, one of:
 *   q_desc (device, fp32, B x d row-major) with descriptors loaded: y is
 *     built on the GPU (step 1); or
 *   q_desc = NULL and y_ids / y_val (device, int32 / fp32, B x k_y
 *     row-major): a precomputed sparse y per query. Ids must lie in
 *     [0, n); a repeated id adds its values.
 * Outputs (each may be NULL when not wanted):
 *   rank_ids, rank_scores (device, int32 / fp32, B x top_k): the top_k items
 *     of x per query, best first, equal scores to the lower id;
 *   x_out (device, fp32, B x n row-major): x = x^s + x^t;
 *   y_ids_out, y_val_out (device, B x k_y): the y that was used;
 *   iters, status (host, int32, B) and relres (host, double, B): per-query
 *     CG iteration count, hd_col_status, and final sqrt(r^T r / y^T y).
 * The call returns when the batch is complete (the stream is synchronised:
 * the CG stopping test reads per-column residuals back to the host).
 * Scalars of CG (dot products, step sizes, residual norms) are double
 * precision on the GPU; vectors are fp32.
 * Errors: HD_ESTATE (no graph, no descriptors for q_desc, rank_r above the
 * loaded r), HD_EINVAL (B < 1, bad options, an id out of range),
 * HD_ENOMEM, HD_EDEVICE.
 */
int hd_query_batch(hd_ctx *ctx, int32_t B, const float *q_desc,
                   const int32_t *y_ids, const float *y_val,
                   const hd_query_opts *opts,
                   int32_t *rank_ids, float *rank_scores, float *x_out,
                   int32_t *y_ids_out, float *y_val_out,
                   int32_t *iters, double *relres, int32_t *status,
                   void *stream);

/*
 * General filters (Appendix A, eq. (2-main)): ranks by x = h(S) y for a
 * polynomial h(x) = sum_{i=0}^{degree} coeffs[i] x^i (for instance a
 * truncated heat kernel or any other series), computed as the spectral term
 * U1 g(L1) U1^T y with g = h - h(0) (eq. (2-aux)) plus the temporal term
 * h(S_r) y, S_r = S - U1 L1 U1^T, by Horner's rule on the deflated operator
 * (degree sparse products, each with the U1 products of the loaded form);
 * rank_r = 0 gives the plain polynomial filter h(S) y. Inputs and outputs as
 * hd_query_batch (q_desc, or y_ids / y_val; rank_ids / rank_scores / x_out
 * device, may be NULL); coeffs: host, degree + 1 values.
 * Errors: as hd_query_batch, HD_EINVAL (degree not in [0, 4096], NULL or
 * non-finite coefficients).
 */
int hd_query_filter(hd_ctx *ctx, int32_t B, const float *q_desc, const int32_t *y_ids, const float *y_val,
                    int32_t degree, const double *coeffs, int32_t rank_r, int32_t k_y, int32_t top_k,
                    int32_t *rank_ids, float *rank_scores, float *x_out, void *stream);

/*
 * Query plans (batching form): the whole query path of hd_query_batch for a
 * fixed batch size B, input kind and options, captured once into a HIP
 * graph and replayed for each batch, so a batch costs one graph launch
 * instead of some ten kernel launches per CG iteration. All max_iter CG
 * iterations are in the graph; once every column has stopped, the later
 * iterations' kernels return at once, so results equal hd_query_batch's
 * (iteration counts, statuses and residuals included). The plan holds its
 * own input and ranking buffers and runs in the context's workspace: it is
 * captured again by itself when that workspace, the loaded data or the
 * launch parameters have changed since. Calls on one context, plans
 * included, must not overlap.
 * input: HD_PLAN_DESCRIPTORS (queries given as B x d fp32 descriptors) or
 * HD_PLAN_Y (B x k_y ids and values of y). The options are those of
 * hd_query_batch; top_k must be >= 1.
 * Errors: as hd_query_batch, HD_EINVAL (input kind, top_k), HD_EDEVICE
 * (capture or instantiation failed).
 */
typedef struct hd_plan hd_plan;
#define HD_PLAN_DESCRIPTORS 0
#define HD_PLAN_Y 1
int hd_plan_create(hd_ctx *ctx, int32_t B, int32_t input, const hd_query_opts *opts, hd_plan **out);

/*
 * Run a plan on stream `stream`: q_desc (device, B x d) for descriptor
 * plans, or y_ids / y_val (device, B x k_y) for y plans, are copied into the
 * plan's buffers, the graph is launched, and the results are written like
 * hd_query_batch's: rank_ids / rank_scores (device, B x top_k, may be NULL),
 * iters / relres / status (host, B, may be NULL). Returns after the stream
 * has finished. Errors: HD_EINVAL (NULL plan or input, a y id outside
 * [0, n) for y plans), HD_EDEVICE.
 */
int hd_plan_run(hd_plan *plan, const float *q_desc, const int32_t *y_ids, const float *y_val,
                int32_t *rank_ids, float *rank_scores, int32_t *iters, double *relres,
                int32_t *status, void *stream);

/* Release a plan (NULL accepted). The context must outlive its plans. */
void hd_plan_destroy(hd_plan *plan);


/*
 * Rank B score vectors (Section 3: decreasing x, equal values to the lower
 * id). x (device, fp32, B x n row-major with row stride ldx >= n elements);
 * ids_out / scores_out (device, B x K). 1 <= K <= min(n, 1024).
 * Runs asynchronously on `stream`. Errors: HD_EINVAL, HD_ENOMEM, HD_EDEVICE.
 */
int hd_rank(hd_ctx *ctx, int32_t B, int64_t n, const float *x, int64_t ldx,
            int32_t K, int32_t *ids_out, float *scores_out, void *stream);

/*
 * hd_rank without any device allocation, for callers that cannot allocate
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc). Same arguments, result and ordering as hd_rank; its scratch is
 * a fixed array of the library on each device (64 MiB, held for the life of
 * the process), so B rows of n items must fit:
 * hd_rank_noalloc_scratch_bytes(B, n, K) <= 64 MiB (about 260 rows of a
 * million items). The array is shared by every call on a device and keeps
 * the last call's contents: calls that overlap on one device (on different
 * streams, or from different threads) race and must not be issued.
 * Errors: HD_EINVAL (as hd_rank, or a size above the fixed scratch),
 * HD_ESTATE (scratch of the context's device not set up), HD_EDEVICE.
 */
int hd_rank_noalloc(hd_ctx *ctx, int32_t B, int64_t n, const float *x, int64_t ldx,
                    int32_t K, int32_t *ids_out, float *scores_out, void *stream);
/* Scratch bytes hd_rank_noalloc needs for B rows of n items (0 for sizes < 1). */
size_t hd_rank_noalloc_scratch_bytes(int32_t B, int64_t n, int32_t K);

/*
 * Memory probes (a measuring aid): the rate the device attains for the
 * access patterns of the query path's memory-bound kernels, by the library's
 * own kernels. mode: 0 = read a buffer of `bytes` once (16-byte loads),
 * 1 = copy it (read + write), 2 = gather whole rows of row_bytes at
 * pseudo-random row ids over the buffer (as many rows as it holds, at
 * least 1 GiB of rows; the sparse product's access to P; a buffer that fits
 * a cache gives that cache's gather rate; the ids are read from an int32
 * array written before the timed launches, 64 per coalesced load, and
 * counted in *bytes_out), 3 = the sparse product's own gathers on
 * the loaded graph without its arithmetic (for every edge, the neighbour's
 * row of an N x row_bytes matrix; `bytes` ignored). row_bytes: 256, 512 or
 * 1024 (modes 2, 3). bytes: a multiple of 4096 in [1 MiB, 64 GiB] (modes
 * 0-2). One warm-up and `reps` timed launches on the null stream; buffers
 * are allocated for the call and freed. Outputs (host): *ms_out, the mean
 * milliseconds per launch; *bytes_out, the bytes one launch reads and
 * writes (mode 3: rows gathered plus the CSR).
 * Errors: HD_EINVAL (arguments), HD_ESTATE (mode 3 with no graph),
 * HD_ENOMEM, HD_EDEVICE.
 */
int hd_probe_memory(hd_ctx *ctx, int32_t mode, int64_t bytes, int32_t row_bytes, int32_t reps,
                    double *ms_out, double *bytes_out);

/* Device bytes currently held by the context (graph, eigenpairs,
 * descriptors, solver workspace). Returns 0 for NULL. */
int64_t hd_device_bytes(const hd_ctx *ctx);

/*
 * Per-kernel timing (a profiling aid). While enabled, every kernel launch of
 * the context is bracketed by a pair of HIP events recorded on the launch
 * stream, and the elapsed times are accumulated per kernel kind at the
 * synchronisation points of hd_query_batch. hd_timing_enable(ctx, 1) turns
 * it on and clears the counters; 0 turns it off. hd_timing_get returns the
 * total milliseconds and the launch count of kernel kind `kind` (0 <=
 * kind < hd_timing_kinds()); hd_timing_name gives its name (NULL if out of
 * range). hd_rank launches are not timed. Errors: HD_EINVAL.
 */
int hd_timing_enable(hd_ctx *ctx, int enable);
/* Like hd_timing_enable(ctx, 1), but only the kernel kinds whose bit
 * (1u << kind) is set in kind_mask are bracketed by events, so the others
 * run without the extra queue packets. */
int hd_timing_enable_kinds(hd_ctx *ctx, uint32_t kind_mask);
int hd_timing_kinds(void);
const char *hd_timing_name(int kind);
int hd_timing_get(const hd_ctx *ctx, int kind, double *total_ms, int64_t *launches);

/*
 * Continuous-batching server. One server keeps a conjugate-gradient solve
 * running over a fixed set of query columns (slots) of the context's graph,
 * eigenpairs and descriptors, which must stay loaded and unchanged while it
 * is open. Requests join free columns between iterations, while other
 * columns are in the middle of their solves, and leave when their column
 * stops: converged (opts.tol), their own iteration cap, y = 0, or breakdown.
 * Each column is an independent recurrence with fixed-order reductions, so a
 * request gets the same result alone or in a full server. The server runs on
 * its own HIP stream. A server is
 * used by one host thread at a time; several servers (e.g. one per
 * database) may run side by side. Calls return when their work is done,
 * except hd_serve_step, which only queues it.
 */
typedef struct hd_server hd_server;

/*
 * Open a server with up to `slots` columns (1..1024) and the options of
 * hd_query_batch (alpha, tol, rank_r, k_y, top_k >= 1; max_iter is the
 * default per-request cap). hbm_budget_bytes > 0 caps the device memory of
 * the server: the column count is the largest power of two >= 64 that fits,
 * and slots is lowered to it (hd_serve_slots reports the result).
 * Errors: HD_EINVAL, HD_ESTATE (no graph, rank_r above the loaded r),
 * HD_ENOMEM (budget below 64 columns, or allocation failure), HD_EDEVICE.
 */
int hd_serve_open(hd_ctx *ctx, int32_t slots, int64_t hbm_budget_bytes,
                  const hd_query_opts *opts, hd_server **out);

/* Device bytes one server column takes on this context with these options
 * (0 for NULL arguments): the unit of hd_serve_open's budget. */
int64_t hd_serve_column_bytes(const hd_ctx *ctx, const hd_query_opts *opts);

/* Column capacity and columns now holding a request (admitted, not polled). */
int hd_serve_slots(const hd_server *srv);
int hd_serve_in_use(const hd_server *srv);

/*
 * Admit up to n requests, in order, into free columns. Input as in
 * hd_query_batch but in HOST memory: q_desc (n x d fp32) or y_ids / y_val
 * (n x k_y). max_iter (host, n entries, >= 0) or NULL for the server default.
 * tickets (host, n) receives an id for each admitted request. Returns the
 * number admitted (0 when no column is free), or a negative hd_status.
 */
int hd_serve_submit(hd_server *srv, int32_t n, const float *q_desc, const int32_t *y_ids,
                    const float *y_val, const int32_t *max_iter, int64_t *tickets);

/* Queue `iters` CG iterations over all columns on the server's stream and
 * return at once (HD_OK or a negative hd_status); the next submit or poll
 * waits for them. Steps of different servers therefore overlap on the GPU. */
int hd_serve_step(hd_server *srv, int32_t iters);

/*
 * Collect up to max_out finished requests and free their columns. Per
 * request (host arrays): tickets, the top_k ranking (ids and scores,
 * max_out x top_k, best first, equal scores to the lower id; each may be
 * NULL), CG iterations, final relative residual and hd_col_status. Returns
 * the number collected, or a negative hd_status.
 */
int hd_serve_poll(hd_server *srv, int32_t max_out, int64_t *tickets, int32_t *ids, float *scores,
                  int32_t *iters, double *relres, int32_t *status);

/*
 * Cancel requests: each of the n tickets (host) that names an admitted
 * request not yet collected by hd_serve_poll has its column stopped after
 * the iterations already queued and freed for the next admission; its
 * results are discarded. The other columns' results do not change (each
 * column is its own recurrence). Tickets that name no such request are
 * ignored. Returns the number of requests cancelled, or a negative
 * hd_status. Errors: HD_EINVAL (NULL server, n < 0, NULL tickets with n > 0),
 * HD_EDEVICE.
 */
int hd_serve_cancel(hd_server *srv, int32_t n, const int64_t *tickets);

/* Release the server's device memory and stream. NULL is accepted. */
void hd_serve_close(hd_server *srv);

#ifdef __cplusplus
}
#endif

#endif /* HD_H */
