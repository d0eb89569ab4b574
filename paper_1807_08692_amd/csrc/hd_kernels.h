// Host-side launchers of the gfx950 kernels (internal to the library).
//
// Layouts used throughout:
//   - graph: CSR with int64 row pointers, int32 columns, fp32 values;
//   - solver vectors (X, R, P, Q, Z): node-major N x ldb fp32, row i holds
//     the ldb query columns of item i; ldb is a power of two >= 64 and the
//     columns B..ldb-1 are padding that stays zero;
//   - eigenvectors U: node-major N x rp (rp = r rounded up to 32, zero
//     padded); coefficient matrices (C, Cl, Cs): rk x ldb;
//   - bfloat16 operands that MFMA kernels stream from memory (the stored U1,
//     item-major and component-major, and the bfloat16 descriptors) are kept
//     in fragment order, see frag_offset;
//   - scores for ranking and similarities: query-major B x ld rows.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace hd {

// Candidate lists of the one-pass top-K (launch_topk_prepare and the
// kernels that take a TopkLists): rows of at least kTopkFuseMin items.
constexpr int64_t kTopkFuseMin = 65536;
constexpr int kTopkChunk = 8192;    // items per candidate list of a row
constexpr int kTopkChunkCap = 256;  // candidates kept per list
struct TopkLists {
    uint64_t *cand;        // [rows][nchunk][kTopkChunkCap] ranking keys
    int32_t *cnt;          // [rows][nchunk] candidates offered to each list
    const uint32_t *thr;   // [rows] order key of the row's threshold
    int nchunk;
};

// Fragment order of an M x K bfloat16 matrix (K a multiple of 32, M padded
// to a multiple of 16 with zero rows): the matrix is cut into 16 x 32 tiles,
// tile (m / 16, k / 32) is stored at tile index (m / 16) kt + k / 32 (kt =
// K / 32 tiles per tile row), and inside a tile as the 64 lanes' operands of
// v_mfma_f32_16x16x32_bf16: lane l = m % 16 + 16 ((k % 32) / 8) holds the
// eight consecutive k of its row at 8 l .. 8 l + 7. A wave then reads a whole
// operand tile as one contiguous kilobyte.
__host__ __device__ inline size_t frag_offset(int64_t m, int64_t k, int64_t kt) {
    const size_t tile = (size_t)(m / 16) * (size_t)kt + (size_t)(k / 32);
    const size_t lane = (size_t)(m % 16) + 16 * (size_t)((k % 32) / 8);
    return (tile * 64 + lane) * 8 + (size_t)(k % 8);
}

// The stored U1 of the matrix-core forms, in fragment order (frag_offset):
// bfloat16 bit patterns (lo = null), two bfloat16 terms hi + lo (lo in the
// same layout), or OCP FP8 E4M3 codes, one byte per element at the same
// element offsets (fp8 = true). The fp8 form carries one fp32 scale per
// component (column of U1); the kernels multiply the codes' values, and the
// scales are applied to the small coefficient matrices (launch_gather_proj,
// launch_reduce_c), never per element.
struct UOperand {
    const void *hi;
    const void *lo;
    bool fp8;
};

// Per-column CG state on the device (all arrays hold ldb entries).
struct CgState {
    double *rho0, *rho, *a, *beta, *relres;
    int32_t *active, *iters, *status;
    int32_t *maxit;      // per-column iteration cap (nullptr: none, the host stops)
    int32_t *nact_part;  // [2][64]: active-column count per 64-column tile,
                         // double buffered by iteration parity
};

// The guard every per-iteration kernel checks: the counts written by the
// previous stopping test (nact) for ntile column tiles.
struct IterGuard {
    const int32_t *nact;
    int ntile;
};

// The last CG iteration's x update (x += a p, the update launch_update_xp
// makes with x_only) carried out by the kernel that reads x next (the
// combine) instead of a pass of its own: element (i, b) of x is taken as
// x + a[b] p(i, b) where a[b] != 0, unless the guard shows every column
// stopped before that iteration. a == nullptr: no fold.
struct XFold {
    const double *a;
    const float *P;  // the search directions, laid out as x (node-major)
    IterGuard g;
};

// Row partition shared by every kernel that writes per-block partial sums:
// block g covers rows [g*rb, min(N, (g+1)*rb)).
struct RowPart {
    int64_t rb;
    int nblk;
};
RowPart make_row_part(int64_t N);

// ---- CG vector kernels (k_cg.hip) ----
hipError_t launch_fill_zero(float *p, size_t n, hipStream_t s);
// zero rows ids[t][u] (t < B, u < ky; ids outside [0, N) skipped) of R and P,
// all ldb columns: before the y scatter when the first CG iteration runs
// with the y row mask instead of full fills of X, R and P
hipError_t launch_zero_yrows(int B, int ky, const int32_t *ids, int64_t N, int ldb, float *R, float *P,
                             hipStream_t s);
// colmap (nullptr = identity): y row t goes to solver column colmap[t];
// rowmask (nullptr = none): bit id of word id / 32 is set for every y id
hipError_t launch_scatter_y(int B, int ky, const int32_t *ids, const float *vals, int64_t N,
                            int ldb, float *R, float *P, int32_t *err, hipStream_t s,
                            const int32_t *colmap = nullptr, uint32_t *rowmask = nullptr);
// part[c] (one row of ldb doubles) = the squared norm of column c of R right
// after the y scatter, from the y ids alone (B y rows of ky ids; colmap as
// in launch_scatter_y, without it columns >= B get 0)
hipError_t launch_ynorm_part(int B, int ky, const int32_t *ids, int64_t N, int ldb, const float *R,
                             double *part, hipStream_t s, const int32_t *colmap = nullptr);
hipError_t launch_cg_init(int B, int ldb, const double *part, int nblk, CgState st, hipStream_t s);
// gamma = the column sums of gpart (nblk rows), plus those of gpart2 (nblk2
// rows) when given. scratch (this and step_b; nullptr = none): 2 x
// kPreSplitRows rows of ldb doubles, where long lists of partial rows are
// first reduced in parallel
constexpr int kPreSplitRows = 64;
hipError_t launch_cg_step_a(int ldb, const double *gpart, int nblk, CgState st, IterGuard g,
                            hipStream_t s, const double *gpart2 = nullptr, int nblk2 = 0,
                            double *scratch = nullptr);
// rowmask (the updates below too; nullptr = none): the first CG iteration
// after launch_zero_yrows, rows outside the mask taken as zero in R and P
// (and X as zero) without reading them; every row is written
hipError_t launch_update_r(int64_t N, int ldb, const float *Q, float *R, RowPart rp,
                           const double *a, double *part, IterGuard g, hipStream_t s,
                           const uint32_t *rowmask = nullptr);
// writes the new per-tile active counts to nact_out
// part == nullptr: the last of a fixed number of products with no residual
// formed (each active column counts it and stops, status MAXITER)
hipError_t launch_cg_step_b(int ldb, const double *part, int nblk, double tol, CgState st,
                            IterGuard g, int32_t *nact_out, hipStream_t s, double *scratch = nullptr);
// width (0 = ldb): only columns [0, width) are updated (row stride ldb);
// x_only: X += a P alone, for the last iteration (P and R untouched)
hipError_t launch_update_xp(int64_t N, int ldb, float *X, float *P, const float *R,
                            const double *a, const double *beta, const int32_t *active,
                            IterGuard g, hipStream_t s, int width = 0,
                            bool x_only = false, const uint32_t *rowmask = nullptr);
// update_xp that also writes the new P as its split transpose (bfloat16
// forms; PT_hi / PT_lo ldb x ldpt in fragment order, ldpt a multiple of 64
// >= N); width as in launch_update_xp. iters (a server's running solve; no
// rowmask): a column's first update (iters 1) overwrites X with a p, and a
// stopped column's P and R are set to zero (its PT with them)
hipError_t launch_update_xp_pt(int64_t N, int ldb, float *X, float *P, float *R,
                               const double *a, const double *beta, const int32_t *active,
                               int64_t ldpt, unsigned short *PTh, unsigned short *PTl, IterGuard g,
                               hipStream_t s, const uint32_t *rowmask = nullptr, int width = 0,
                               const int32_t *iters = nullptr);
hipError_t launch_cg_final(int ldb, CgState st, hipStream_t s);
// colmap (nullptr = identity, B columns of ldb): y row t -> column colmap[t]
// U: fp32 item-major N x rp (fmt = 0), bfloat16 bit patterns in fragment
// order over N x rp (fmt = 1, value U + U_lo when U_lo is not null: the
// two-term storage form) or FP8 E4M3 codes in fragment order (fmt = 2) with
// uscale[k] the scale of component k. c = U1^T y is exact for the stored
// U1 (codes times scales); with uscale, Cs and Cl are written pre-multiplied
// by uscale (the coefficients of the codes in U1 Cs and U1 Cl) while Dg uses
// c itself.
hipError_t launch_gather_proj(int B, int ky, const int32_t *ids, const float *vals, int64_t N,
                              const void *U, const void *U_lo, int fmt, int rp, int rk, int r_use,
                              const double *lam, double alpha, int ldb, float *Cs, float *Cl,
                              hipStream_t s, const int32_t *colmap = nullptr, const double *gv = nullptr,
                              double *Dg = nullptr, const float *uscale = nullptr);
// P = c R + qs Q over n floats (polynomial filter step); qs = 0 does not read Q
hipError_t launch_filter_axpy(float *P, const float *R, const float *Q, size_t n, double c, double qs,
                              hipStream_t s);

// ---- continuous batching (columns joining and leaving a running solve) ----
// zero columns cols[0..ncols) of X, R and P
hipError_t launch_zero_cols(int64_t N, int ldb, float *X, float *R, float *P, const int32_t *cols,
                            int ncols, hipStream_t s);
// start the CG recurrence of columns cols[0..ncols) from the R^T R partials:
// rho0 = rho = y^T y, iteration 0, cap maxit[t] (written to st.maxit)
hipError_t launch_init_cols(int ldb, const double *part, int nblk, CgState st, const int32_t *cols,
                            const int32_t *maxit, int ncols, hipStream_t s);
// columns cols[0..ncols) stop: inactive from now on (their vectors untouched)
hipError_t launch_cancel_cols(CgState st, const int32_t *cols, int ncols, hipStream_t s);
// Xc (N x ldc node-major) and Csc (rk x ldc) = the columns cols[0..ncols) of X and Cs;
// iters (nullptr = none): columns with no iteration done give x = 0
hipError_t launch_gather_cols(int64_t N, int ldb, const float *X, const float *Cs, int rk,
                              const int32_t *cols, int ncols, int ldc, float *Xc, float *Csc,
                              hipStream_t s, const int32_t *iters = nullptr);

// ---- persistent CG for narrow batches (k_persist.hip): node-major N x W
//      vectors, W a power of two in 1..64; plain CG, or with fp32 U1
//      (rp = row stride, rk components, W <= 16, rk <= 1024) ----
bool persist_width_ok(int W, int rk);
size_t persist_lds_bytes(int W, int rk);
// co-resident grid for width W and rk components on N rows (0: not possible)
int persist_grid(int W, int rk, int64_t N);
// Runs every CG iteration (up to max_iter, stopping test tol per column):
// on entry X = 0, R = P = y, Cl = L1 U1^T y (hybrid), yn[c] = y^T y; on exit
// X = the temporal term and st the per-column results (relres by
// launch_cg_final). sync_words: 4 zeroed words; err[1] is set if a grid
// barrier wait ran past spin_limit (the kernel then ends early).
hipError_t launch_cg_persist(int W, int grid, int64_t N, const int64_t *rowptr, const int32_t *col,
                             const float *val, const float *U, int rp, int rk, int r_use, const double *lam,
                             double alpha, float *X, float *R, float *P, float *Q, float *Cl, float *Cpart,
                             double *gpart, double *rpart, const double *yn, CgState st, int B, int max_iter,
                             double tol, unsigned *sync_words, long long spin_limit, int32_t *err,
                             hipStream_t s);
// x[b][i] = (U1 Cs)[i][b] + X[i][b], b < B, X narrow (N x W), Cs rk x W
hipError_t launch_combine_narrow(int W, int64_t N, int B, const float *U, int rp, int rk, const float *Cs,
                                 const float *X, float *x, int64_t ldx, hipStream_t s);

// ---- sparse product (k_spmm.hip) ----
// Q = (Zs - alpha * S P) / (1 - alpha); gpart[g][c] = sum over the rows of
// block g of P[i][c] * Q[i][c] (double). With rowmask, neighbour rows whose
// bit is clear (all zero in P) are not gathered; the result is the same. The launchers that take a width
// (0 = ldb; a multiple of 64) compute only columns [0, width) of vectors of
// row stride ldb.
hipError_t launch_spmm(int64_t N, const int64_t *rowptr, const int32_t *col, const float *val,
                       const float *P, const float *Zs, float *Q, int ldb, double alpha,
                       RowPart rp, double *gpart, IterGuard g, hipStream_t s, int cpl = 0,
                       int width = 0, const uint32_t *rowmask = nullptr, int bands = 1,
                       const int32_t *cut = nullptr);
// valid source-band counts of launch_spmm (1, 2, 4, 8)
bool band_param_ok(int v);
// cut[8 i + b - 1], b = 1..8: the number of row i's edges whose neighbour id
// is below b N / 8 (host; rows with strictly increasing columns)
void build_band_cuts(int64_t N, const int64_t *rowptr, const int32_t *col, int32_t *cut);

// ---- eigenvector products on MFMA (k_ugemm.hip) ----
// Number of row chunks of the split-K product U^T P.
int ut_p_chunks(int64_t N, int64_t *rows_per_chunk);
// Cpart[c] = U[chunk c]^T P[chunk c]  (rk x ldb per chunk)
hipError_t launch_ut_p(int64_t N, const float *U, int rp, int rk, const float *P, int ldb,
                       float *Cpart, IterGuard g, hipStream_t s);
// Cl = lambda .* sum_c Cpart[c]   (rows k >= r_use zeroed); with Dg also
// Dg = alpha / (1 - alpha) lambda .* (sum_c Cpart[c])^2 (double, rk x ldb):
// the eigenvector part of P^T Q when the correction follows the sparse product
// With uscale (the fp8 form: Cpart holds the products of the codes), the
// sum of component k is first multiplied by uscale[k] (giving U1^T P), and Cl
// is written pre-multiplied by uscale[k] once more (the coefficient of the
// codes in U1 Cl).
hipError_t launch_reduce_c(int nchunk, const float *Cpart, int rk, int ldb, const double *lam,
                           int r_use, float *Cl, IterGuard g, hipStream_t s, double *Dg = nullptr,
                           double alpha = 0.0, const float *uscale = nullptr);
// Z = P + alpha * U Cl
hipError_t launch_u_c(int64_t N, const float *U, int rp, int rk, const float *Cl, int ldb,
                      const float *P, double alpha, float *Z, IterGuard g, hipStream_t s);
// x[b][i] = (U Cs)[i][b] + X[i][b] for b < B, i < N   (x row stride ldx)
// gate (nullptr = none): every block returns at once while *gate == 0
hipError_t launch_combine(int64_t N, int B, const float *U, int rp, int rk, const float *Cs,
                          int ldb, const float *X, float *x, int64_t ldx, hipStream_t s,
                          const int32_t *gate = nullptr, const XFold *fold = nullptr);  // fold: rk = 0 only

// ---- bfloat16 storage form of the eigenvector and descriptor products
//      (k_ugemm_bf16.hip); bf16 values are passed as their 16-bit patterns.
//      The stored U1 (UOperand: one or two bfloat16 terms, or FP8 codes) and
//      the descriptors are in fragment order (frag_offset) ----
// CT_hi / CT_lo (ldb x rk, bf16, fragment order; rk a multiple of 32) = hi /
// lo split of C^T (C: rk x ldb fp32).
// A null g.nact disables the iteration guard.
hipError_t launch_split_t(const float *C, int rk, int ldb, unsigned short *CT_hi,
                          unsigned short *CT_lo, IterGuard g, hipStream_t s);
// PT_hi / PT_lo (ldb x ldpt, bf16, fragment order over items, zero past N) =
// hi / lo split of P^T (P: N x ldb fp32 node-major); ldpt a multiple of 64.
hipError_t launch_split_pt(int64_t N, int ldb, const float *P, int64_t ldpt, unsigned short *PTh,
                           unsigned short *PTl, IterGuard g, hipStream_t s, int width = 0);
// Columns cols[0..m) admitted into a running solve, their P set to y (the
// k_y rows ids[t * ky ..] of column cols[t], zero elsewhere): the part of
// PT_hi / PT_lo of the columns zcols[0..nz) (those whose PT may not be zero)
// is zeroed, then every admitted column's is written from P at its y rows,
// as launch_split_pt would write it.
hipError_t launch_pt_admit(int m, int ky, const int32_t *ids, const int32_t *cols, const int32_t *zcols, int nz,
                           int64_t N, int ldb, const float *P, int64_t ldpt, unsigned short *PTh,
                           unsigned short *PTl, hipStream_t s);
// Cpart[c] = U[chunk c]^T P[chunk c], U given component-major (UT: the
// rp x ldut matrix in fragment order, zero past N) and P as its split
// transpose (PT_hi / PT_lo, pitch ldut)
hipError_t launch_ut_p_bf16(int64_t N, UOperand UT, int64_t ldut, int rk, const unsigned short *PTh, const unsigned short *PTl,
                            int ldb, float *Cpart, IterGuard g, hipStream_t s, int nt = 0,
                            int width = 0);
// Z = P + alpha U Cl, U item-major (N x rp in fragment order, rows padded to
// a multiple of 16), Cl given as split transpose
hipError_t launch_u_c_bf16(int64_t N, UOperand U, int rp, int rk,
                           const unsigned short *CT_hi, const unsigned short *CT_lo, int ldb,
                           const float *P, double alpha, float *Z, IterGuard g, hipStream_t s,
                           int nt = 0);
// With Qs = (P - alpha S P) / (1 - alpha) (launch_spmm with Zs = P): the
// residual update r -= a (Qs + alpha / (1 - alpha) U Cl) (Cl as split
// transpose), and part[g][c] = sum over the rows of 128-row block g of the
// new r^2 (uc_update_r_blocks(N) rows of ldb doubles). iters / maxit (a
// server's running solve; no rowmask): a column whose cap ends it in this
// iteration (iters + 1 >= maxit) has its new r counted in r^2 but stored as
// zero
int uc_update_r_blocks(int64_t N);
hipError_t launch_uc_update_r_bf16(int64_t N, UOperand U, int rp, int rk, const unsigned short *CT_hi, const unsigned short *CT_lo, int ldb,
                                   const float *Qs, double alpha, float *R, const double *a, double *part,
                                   IterGuard g, hipStream_t s, int nt = 0, int width = 0,
                                   const uint32_t *rowmask = nullptr, const int32_t *iters = nullptr,
                                   const int32_t *maxit = nullptr);
// x[b][i] = (U Cs)[i][b] + X[i][b], Cs given as split transpose
// n-tiles per wave launch_combine_bf16 uses for width ldb and requested
// value req (0 = default); the fold is not available with 4
int combine_nt(int ldb, int req);
// tl (one-pass top-K): candidates to the lists, x not written; gate as in
// launch_combine
hipError_t launch_combine_bf16(int64_t N, int B, UOperand U, int rp, int rk,
                               const unsigned short *CT_hi, const unsigned short *CT_lo, int ldb,
                               const float *X, float *x, int64_t ldx, hipStream_t s, int nt = 0,
                               const TopkLists *tl = nullptr, const int32_t *gate = nullptr,
                               const XFold *fold = nullptr);
// Tile parameters: a requested value (0 = default) is valid for width ldb
// when it is one of 1, 2, 4 and divides the width in 64-column units.
bool tile_param_ok(int v, int ldb);
// sim[b][j] = q[b] . V[j], V stored bf16 (N x ldv, fragment order), or as
// FP8 E4M3 codes in the same order (vscale != null: row j's value is
// vscale[j] times its codes); qsplit: scratch for 2 x sim_qsplit_rows(B) x
// ldv bf16 (the hi / lo parts of q)
inline int sim_qsplit_rows(int B) { return (B + 63) / 64 * 64; }
// tl (one-pass top-K): candidates to the lists, sim not written; gate: every
// block returns at once while *gate == 0; split_q = false reuses the split
// of q already in qsplit (the same q, B and d)
hipError_t launch_sim_bf16(int64_t N, int B, int d, const float *q, const void *V,
                           int ldv, unsigned short *qsplit, float *sim, int64_t lds, hipStream_t s,
                           const float *vscale = nullptr, const TopkLists *tl = nullptr,
                           const int32_t *gate = nullptr, bool split_q = true);

// ---- similarity product for the observation vector (k_sim.hip) ----
// sim[b][j] = sum_t q[b][t] V[j][t]  (q: B x d, row stride d; V: N x ldv)
hipError_t launch_sim(int64_t N, int B, int d, const float *q, const float *V, int ldv,
                      float *sim, int64_t lds, hipStream_t s);

// ---- top-K selection (k_topk.hip) ----
constexpr int kTopkMax = 1024;
// Bytes of scratch for selecting K of n in B rows.
size_t topk_scratch_bytes(int B, int64_t n, int K);
// ids/scores (B x K): the K largest x per row, best first, equal values to
// the lower id. transform = 1 writes max(0, s)^3 in place of the score.
hipError_t launch_topk(int B, int64_t n, const float *x, int64_t ldx, int K, void *scratch,
                       int32_t *ids, float *scores, int transform, hipStream_t s);

// ---- one-pass top-K: the filter fused into the kernel that produces the
//      scores (rows of n >= kTopkFuseMin items; same scratch as launch_topk).
// The scores of a fixed sample of each row (items t * stride, t < m, see
// topk_sample) set the row's threshold (launch_topk_prepare); the score
// kernel, given the TopkLists, appends every score at or above it to the
// row's candidate lists and writes no score matrix; launch_topk_select_lists
// sorts the lists. A row whose lists overflow or hold fewer than K is
// flagged and left unwritten: a second launch of the score kernel gated on
// topk_fallback_gate (its blocks return at once when no row is flagged)
// writes the score matrix, and launch_topk_fallback selects the flagged rows
// exactly from it. The result is the one launch_topk gives on the same scores.
void topk_sample(int64_t n, int64_t *stride, int64_t *m);
TopkLists topk_lists(void *scratch, int B, int64_t n);
const int32_t *topk_fallback_gate(void *scratch, int B, int64_t n);
// thresholds from the sample scores: value t of row b at S[b * ld_row + t * ld_item];
// also empties the lists and clears the flags
hipError_t launch_topk_prepare(int B, int64_t n, const float *S, int64_t ld_row, int64_t ld_item, int K,
                               void *scratch, hipStream_t s);
hipError_t launch_topk_select_lists(int B, int64_t n, int K, void *scratch, int32_t *ids, float *scores,
                                    int transform, hipStream_t s);
hipError_t launch_topk_fallback(int B, int64_t n, const float *x, int64_t ldx, int K, void *scratch,
                                int32_t *ids, float *scores, int transform, hipStream_t s);
// candidates of the scores x[b][i] = X[i][b] (node-major X, b < B <= ldb)
hipError_t launch_topk_emit_nm(int64_t n, int B, int ldb, const float *X, TopkLists tl, hipStream_t s,
                               const XFold *fold = nullptr);
// the sample's rows: fragment-order matrices (ld a multiple of 32, elem_bytes
// 2 or 1; dst is m rounded up to 16 rows, zero past m) and row-major rows
hipError_t launch_sample_frag(int64_t m, int64_t stride, int64_t ld, const void *src, void *dst, int elem_bytes,
                              hipStream_t s);
// fold (ld = the solver width): the sampled rows of x with the fold applied
hipError_t launch_sample_rows(int64_t m, int64_t stride, int ld, const float *src, float *dst, hipStream_t s,
                              const XFold *fold = nullptr);

// ---- SHybrid: sparsified U1 (k_sparse_u.hip). U~ by item (CSR rptr / rcol /
//      rval, N rows) and by component (CSC cptr / crow / cval, rk columns) ----
hipError_t launch_sp_utp(int rk, int r_use, const int64_t *cptr, const int32_t *crow, const float *cval,
                         const float *P, int ldb, const double *lam, float *Cl, IterGuard g, hipStream_t s);
hipError_t launch_sp_uc(int64_t N, const int64_t *rptr, const int32_t *rcol, const float *rval,
                        const float *Cl, int ldb, const float *P, double alpha, float *Z, IterGuard g,
                        hipStream_t s);
hipError_t launch_sp_gather_proj(int B, int ky, const int32_t *ids, const float *vals, int64_t N,
                                 const int64_t *rptr, const int32_t *rcol, const float *rval, int rk,
                                 int r_use, const double *lam, double alpha, int ldb, float *Cs, float *Cl,
                                 hipStream_t s, const int32_t *colmap = nullptr, const double *gv = nullptr);
hipError_t launch_sp_combine(int64_t N, int B, const int64_t *rptr, const int32_t *rcol, const float *rval,
                             const float *Cs, int ldc, const float *X, float *x, int64_t ldx, hipStream_t s);

// ---- top-r eigensolver blocks (k_eig.hip): N x m item-major, double ----
hipError_t launch_eig_rand(int64_t N, int m, uint64_t seed, double *X, hipStream_t s);
// Out = a S Y1 + b Y1 + c Y0 (Y0 may be null); m a multiple of 64
hipError_t launch_eig_cheb(int64_t N, const int64_t *rowptr, const int32_t *col, const float *val, int m,
                           const double *Y1, const double *Y0, double *Out, double a, double b, double c,
                           hipStream_t s);
hipError_t launch_eig_resid(int64_t N, int m, const double *SX, const double *X, const double *w, int64_t rb,
                            int nblk, double *part, hipStream_t s);
hipError_t launch_eig_extract(int64_t N, int m, int r, const double *X, float *U, hipStream_t s);
// ---- FP64 matrix-core products of the eigensolver blocks (k_eig_gemm.hip);
//      m a multiple of 64 ----
// row chunks of the split Gram product (Gpart holds gram_chunks(N) m x m)
int64_t gram_chunks(int64_t N);
// G (m x m, row-major) = A^T B, A and B item-major N x m
hipError_t launch_gram(int64_t N, int m, const double *A, const double *B, double *Gpart, double *G,
                       hipStream_t s);
// Y = X Z (item-major N x m), Z column-major m x m with leading dimension ldz; Y != X
hipError_t launch_rotate(int64_t N, int m, const double *X, const double *Z, int ldz, double *Y, hipStream_t s);

}  // namespace hd
