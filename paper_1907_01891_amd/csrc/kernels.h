// Host-side launchers of the libctqr kernels (internal interface).
#pragma once
#include "common.h"

// ---- gemm.hip --------------------------------------------------------------
// Products launched from this host thread with at most gemm_narrow_max()
// output columns use the 128 x 32 output tile (0: never).
int gemm_narrow_max();
void gemm_set_narrow_max(int n);
int gemm_tn_splits(int M, int N, int K);
size_t gemm_tn_partial_elems(int M, int N, int K);
// force_splits > 0 fixes the number of K splits (the partial buffer must hold
// them, else CTQR_ENOMEM): products over different column ranges of one
// matrix then sum every output in the same order.  bf16 (FP32 operands,
// 128-wide tiles): 1 = operands rounded to bf16 while staged, BF16 MFMA with
// FP32 accumulation (gemm_nn: the trailing update, kind 1, only); 2 (split
// parts) is refused with CTQR_EINVAL: gemm_tn_bf16x3 / gemm_nn_bf16x3 below.
// tri (square A, M = K): A(k, m) is zero for k < m (1: A is the transpose of
// an upper triangular block) or for k > m (2: upper triangular), and the
// steps of exact zeros are skipped.
template <typename T>
ctqr_status gemm_tn(int M, int N, int K, const T *A, int64_t lda, int amask, const T *B,
                    int64_t ldb, int bmask, T alpha, T beta, T *Out, int64_t ldo, T *part,
                    size_t part_elems, const int *skip, hipStream_t st, int force_splits = 0,
                    int bf16 = 0, int tri = 0);
// W2 = Tt^T (A^T B) for a product of at most 32 rows (the update by a 32-wide
// inner panel, Tt its 32 x 32 factor): A^T B as gemm_tn (written to Out when
// it is not split over K), then one launch that finishes the split-K sum and
// multiplies by Tt^T.
template <typename T>
ctqr_status gemm_tn_tprod(int M, int N, int K, const T *A, int64_t lda, int amask, const T *B, int64_t ldb,
                          const T *Tt, int64_t ldt, T *Out, int64_t ldo, T *W2, int64_t ldw, T *part,
                          size_t part_elems, hipStream_t st);
template <typename T>
ctqr_status gemm_nn(int M, int N, int K, const T *A, int64_t lda, int amask, const T *B,
                    int64_t ldb, T alpha, T *C, int64_t ldc, const int *skip, hipStream_t st,
                    int kind = 0, int accum = 1, int bf16 = 0);
// `batch` products C_b (+)= alpha A_b B_b (A not a Householder block), operand
// b at A + b bsa, B + b bsb, C + b bsc, in one launch (accum as gemm_nn).
template <typename T>
ctqr_status gemm_nn_batched(int M, int N, int K, const T *A, int64_t lda, int64_t bsa, const T *B, int64_t ldb,
                            int64_t bsb, T alpha, T *C, int64_t ldc, int64_t bsc, int batch, int accum,
                            hipStream_t st);
// C += alpha A B (A not a Householder block), split over K into part when the
// output has too few tiles to fill the chip.
template <typename T>
ctqr_status gemm_nn_split(int M, int N, int K, const T *A, int64_t lda, const T *B, int64_t ldb, T alpha,
                          T *C, int64_t ldc, T *part, size_t part_elems, const int *skip, hipStream_t st);

// Split-BF16 trailing update C += alpha V W' (V: M x K Householder block,
// column-major lda; W': K x N, column-major ldw).  bf16x3_split writes both
// operands' high and low bf16 parts to `split` (bf16x3_split_elems(m, n, nb)
// elements cover any M <= m, N <= n, K <= nb); gemm_nn_bf16x3 then forms the
// product from them, three BF16 products per pair with FP32 accumulation.
// kind (1 or 2) only selects the kernel instance, so that profiles tell the
// trailing update (1) from the update of a pair's second block column (2).
size_t bf16x3_split_elems(int64_t m, int64_t n, int nb);
// householder = false splits a plain M x K operand (a block of R).
ctqr_status bf16x3_split(int M, int N, int K, const float *V, int64_t lda, const float *W, int64_t ldw,
                         __bf16 *split, size_t split_elems, hipStream_t st, bool householder = true,
                         const int *skip = nullptr);
ctqr_status gemm_nn_bf16x3(int M, int N, int K, float alpha, float *C, int64_t ldc, const __bf16 *split,
                           size_t split_elems, hipStream_t st, const int *skip = nullptr, int kind = 1);
// The same pieces with caller-placed parts: an M x K operand to row-major
// parts (row stride ldp, rows up to rows_pad, a multiple of 128, zero), a
// K x N operand to column-major parts (column stride ldp, columns up to
// cols_pad, a multiple of 128, zero), both zero for k in [K, ldp); and the
// product C += alpha A B from such parts.
ctqr_status bf16x3_split_rows(int M, int K, const float *V, int64_t lda, bool householder, __bf16 *hi, __bf16 *lo,
                              int ldp, int rows_pad, hipStream_t st, const int *skip = nullptr);
ctqr_status bf16x3_split_cols(int K, int N, const float *W, int64_t ldw, __bf16 *hi, __bf16 *lo, int ldp,
                              int cols_pad, hipStream_t st, const int *skip = nullptr);
ctqr_status gemm_nn_bf16x3_parts(int M, int N, int K, float alpha, float *C, int64_t ldc, const __bf16 *ah,
                                 const __bf16 *al, int64_t lda_p, const __bf16 *bh, const __bf16 *bl, int64_t ldb_p,
                                 hipStream_t st, const int *skip = nullptr);

// Split-BF16 reduction Out = alpha V^T B + beta Out (V: K x M Householder
// block, M <= 256): bf16x3_split_vt writes V's high and low bf16 parts once to
// `vt` (bf16x3_vt_elems(m, nb) elements cover any K <= m, M <= nb);
// gemm_tn_bf16x3 then forms the products with B split while staged, split
// over K by the same rule as gemm_tn.
size_t bf16x3_vt_elems(int64_t m, int nb);
ctqr_status bf16x3_split_vt(int rows, int kc, const float *V, int64_t lda, __bf16 *vt, size_t vt_elems,
                            hipStream_t st, bool householder = true, const int *skip = nullptr);
// gram_cols: the output's first gram_cols columns are the Gram V^T V (B's
// first columns being V itself); its tiles wholly below the diagonal are not
// formed (only the diagonal and upper blocks of a Gram are read).
ctqr_status gemm_tn_bf16x3(int M, int N, int K, const __bf16 *vt, size_t vt_elems, const float *B, int64_t ldb,
                           int bmask, float alpha, float beta, float *Out, int64_t ldo, float *part,
                           size_t part_elems, const int *skip, hipStream_t st, int force_splits, int gram_cols = 0);

// ---- panel_qr.hip ----------------------------------------------------------
constexpr int PANEL_XCH_STRIDE = 40;   // doubles per workgroup per exchange buffer (two buffers)
int panel_rows_per_wg(int mrem, int ncu);
int panel_max_rows_per_wg();       // FP64 slab
int panel_max_rows_per_wg_f32();   // FP32 slab (FP32 storage only)
ctqr_status panel_setup(int max_rows);
template <typename TS>
ctqr_status panel_qr(TS *A, int64_t lda, int m, int r0, int w, double *tau, double *part,
                     double *part2, double *gram_part, double *gram, TS *Tin, bool want_t, unsigned *bar,
                     ctqr_info *info, int ncu, hipStream_t st);
// The panel's T (PW x PW, leading dimension PW) is stored to Tin by the panel
// kernel itself: by the reconstruction route, or, when want_t is set, after
// the column route from the summed Gram V^T V (gram: PANEL_GRAM_ELEMS doubles).
constexpr int PANEL_GRAM_ELEMS = 32 * 32;
template <typename TG, typename TT>
ctqr_status tbuild(int nb, const TG *G, int64_t ldg, const double *tau, TT *T, int64_t ldt, double *Tw,
                   hipStream_t st, const double *skip = nullptr);

// ---- trsm.hip --------------------------------------------------------------
constexpr int TRSM_BASE = 256;  // diagonal block inverted directly
constexpr int TRSM_BIG = 2048;  // diagonal block of the block substitutions
size_t trinv_elems(int n);      // Rinv: TRSM_BIG x round_up(n, TRSM_BIG)
size_t trinv_tmp_elems();
template <typename T>
ctqr_status trinv_blocks(int n, const T *R, int64_t ldr, T *Rinv, T *tmp, ctqr_info *info,
                         hipStream_t st);
// the diagonal blocks starting in columns [c0, c1) only (block-size multiples)
template <typename T>
ctqr_status trinv_blocks_range(int n, int c0, int c1, const T *R, int64_t ldr, T *Rinv, T *tmp,
                               hipStream_t st);
// Split-BF16 parts for the wide substitutions: r holds R's off-diagonal
// blocks split once by trsm_split_r (trsm_rparts_elems(n) elements), x the
// right-hand side's parts of one product (trsm_xparts_elems(S)).  Given
// (FP32 R, at least TRSM_SPLIT_MIN_SLICES slices), the off-diagonal block
// products of the right-looking substitutions run on split-BF16 MFMA.
constexpr int TRSM_SPLIT_MIN_SLICES = 128;
struct TrsmParts {
    const __bf16 *r;
    __bf16 *x;
};
size_t trsm_rparts_elems(int64_t n);
size_t trsm_xparts_elems(int S);
ctqr_status trsm_split_r(int n, const float *R, int64_t ldr, __bf16 *parts, hipStream_t st);
template <typename T>
ctqr_status trsm_upper(int n, int S, const T *R, int64_t ldr, const T *Rinv, T *C, int64_t ldc,
                       T *X, int64_t ldx, T *part, size_t part_elems, const int *skip, hipStream_t st,
                       const TrsmParts *rp = nullptr);
template <typename T>
ctqr_status trsm_upper_trans(int n, int S, const T *R, int64_t ldr, const T *Rinv, T *C, int64_t ldc,
                             T *Y, int64_t ldy, T *part, size_t part_elems, const int *skip,
                             hipStream_t st, const TrsmParts *rp = nullptr);
// out[k] = A(k, k) for k in [c0, c1)
template <typename T>
ctqr_status diag_copy(int c0, int c1, const T *A, int64_t lda, T *out, hipStream_t st);
// column-block ranges of the substitutions (right-looking R X = C over the
// blocks starting in [c_lo, c_hi), last first; left-looking R^T Y = C, first
// first); each step reads only its own column block of R
template <typename T>
ctqr_status trsm_upper_cols(int n, int S, const T *R, int64_t ldr, const T *Rinv, T *C, int64_t ldc, T *X,
                            int64_t ldx, int c_lo, int c_hi, T *part, size_t part_elems, const int *skip,
                            hipStream_t st);
template <typename T>
ctqr_status trsm_upper_trans_cols(int n, int S, const T *R, int64_t ldr, const T *Rinv, T *C, int64_t ldc, T *Y,
                                  int64_t ldy, int c_lo, int c_hi, T *part, size_t part_elems, const int *skip,
                                  hipStream_t st);
template <typename T>
ctqr_status rdiag_check(int n, const T *R, int64_t ldr, double *scratch, ctqr_info *info,
                        hipStream_t st);

// ---- siddon.hip ------------------------------------------------------------
ctqr_status siddon_build(const ctqr_geometry *g, int dtype, void *A, int64_t lda, ctqr_sparse *sp,
                         void *work, size_t work_bytes, ctqr_info *info, hipStream_t st);
size_t siddon_workspace(const ctqr_geometry *g);
// B = J X with Joseph's projector (m x S and n x S, column-major FP64)
ctqr_status joseph_project(const ctqr_geometry *g, int S, const double *X, int64_t ldx, double *B, int64_t ldb,
                           hipStream_t st);

// ---- quality.hip -------------------------------------------------------------
// out[s] = PSNR, out[S + s] = mean SSIM of X[:, s] against Xref[:, s]
ctqr_status image_quality(int side, int S, const double *Xref, int64_t ldr, const double *X, int64_t ldx,
                          double data_range, double *out, hipStream_t st);
// columns [c0, c1) of the dense A (FP64 or FP32) from the CSC copy
ctqr_status sparse_to_dense_cols(const ctqr_sparse *sp, int dtype, int c0, int c1, void *A, int64_t lda,
                                 hipStream_t st);

// ---- sparse.hip / util ------------------------------------------------------
// y[i, :] = alpha * sum_k val[k] x[idx[k], :] + beta * y[i, :] for rows i of a
// compressed matrix (CSR or CSC), x and y row-major (slice index fastest).
// tside > 0 (rows = tside^2, tside a multiple of 16): the rows are the pixels
// of a square image and the wide forms visit them in 16 x 16 tiles (same
// results, better L2 reuse of the gathered rows).
ctqr_status spmm_rowmajor(int64_t rows, int S, const int64_t *ptr, const int32_t *idx,
                          const double *val, double alpha, const double *x, double beta,
                          const double *y_in, double *y, const int *skip, hipStream_t st, int tside = 0);
// tside for the pixels of A^T: the image side when n is the square of a
// multiple of 16 (the column layout of ctqr_build_system_matrix), else 0.
int pixel_tile_side(int64_t n);
ctqr_status spmm_colmajor(int64_t rows, int64_t cols, int S, const int64_t *ptr, const int32_t *idx,
                          const double *val, double alpha, const double *X, int64_t ldx,
                          double beta, double *Y, int64_t ldy, hipStream_t st);
// dst (rows x S, column-major, ld) <-> row-major copies with type conversion
template <typename TD, typename TSRC>
ctqr_status cm_to_rm(int64_t rows, int S, const TSRC *src, int64_t lds, TD *dst, const int *skip,
                     hipStream_t st);
template <typename TD, typename TSRC>
ctqr_status rm_to_cm(int64_t rows, int S, const TSRC *src, TD *dst, int64_t ldd, const int *skip,
                     hipStream_t st);
// the first S of the ss slices of a row-major FP64 array, column-major
ctqr_status rm_to_cm_sub(int64_t rows, int ss, int S, const double *src, double *dst, int64_t ldd,
                         hipStream_t st);
template <typename TD, typename TSRC>
ctqr_status copy_cm(int64_t rows, int S, const TSRC *src, int64_t lds, TD *dst, int64_t ldd,
                    hipStream_t st);
ctqr_status fill_u32(unsigned *p, int64_t n, unsigned v, hipStream_t st);
ctqr_status fill_f64(double *p, int64_t n, double v, hipStream_t st);
ctqr_status info_reset(ctqr_info *info, hipStream_t st);
// Refinement step: x += d (row-major x FP64, column-major d of type TD),
// per-slice max|d| and max|x| into dmax/xmax (bit patterns, atomic max); xs
// (row-major like x, or null) receives x before the update.
template <typename TD>
ctqr_status refine_update(int64_t n, int S, double *x, const TD *d, int64_t ldd,
                          unsigned long long *dmax, unsigned long long *xmax, double *xs, const int *skip,
                          hipStream_t st);
// Converged when the relative update is <= tol; stall_limit consecutive
// non-contracting updates, or max_iters, end it with CTQR_NOT_CONVERGED.
// Also records the best iterate so far (hist[2..7]).
// The best iterate is judged by smax (per-slice max |A^T (b - A x)| of the
// iteration's starting iterate, from slice_absmax) relative to s0, the first
// iteration's values (written at it = 0).
ctqr_status refine_check(int S, unsigned long long *dmax, unsigned long long *xmax, unsigned long long *smax,
                         double *s0, double tol, int it, int max_iters, int stall_limit, double *hist, int *done,
                         ctqr_info *info, hipStream_t st);
// smax[s] = max(smax[s], max_r |x[r, s]|) for a row-major rows x S array
ctqr_status slice_absmax(int64_t rows, int S, const double *x, unsigned long long *smax, const int *skip,
                         hipStream_t st);
// xbest = xs (count doubles) when the last refine_check found a new smallest update.
ctqr_status refine_keep(int64_t count, const double *xs, double *xbest, const double *hist, hipStream_t st);
// After CTQR_NOT_CONVERGED: x = xbest unless the smallest update was the last one.
ctqr_status refine_select(int64_t count, double *x, const double *xbest, const double *hist, ctqr_info *info,
                          hipStream_t st);

// ---- refine.hip (conjugate-gradient form of the refinement) -----------------
constexpr int PCG_DOT_BLOCKS = 256;
size_t slice_dot_partial_elems(int S);
// out[s] = sum_i x[i, s] y[i, s] (row-major, deterministic two-pass sum)
ctqr_status slice_dot(int64_t rows, int S, const double *x, const double *y, double *partial, double *out,
                      const int *skip, hipStream_t st);
ctqr_status pcg_beta(int S, int first, const double *sz, const double *szp, double *gamma, double *beta,
                     const int *skip, hipStream_t st);
ctqr_status pcg_alpha(int S, const double *gamma, const double *qq, double *alpha, const int *skip,
                      hipStream_t st);
ctqr_status pcg_direction(int64_t rows, int S, const double *z, const double *beta, double *p, const int *skip,
                          hipStream_t st);
ctqr_status pcg_step(int64_t rows, int S, double *x, const double *p, const double *alpha,
                     unsigned long long *dmax, unsigned long long *xmax, double *xs, const int *skip,
                     hipStream_t st);

// ---- cond.hip (condition-number estimate) ------------------------------------
// Column-major rows x S vectors (cond_start: row-major when ldx = 0):
// counter-hashed start values in [-1, 1),
// FP64 column dot products (deterministic), scaling to unit norm, and the
// running maximum of Rayleigh quotients (est[slot]); cond_finish writes
// [sigma_max, sigma_min, kappa] from est[0] (A^T A) and est[1] ((R^T R)^-1).
template <typename T>
ctqr_status cond_start(int64_t rows, int S, T *x, int64_t ldx, uint64_t seed, hipStream_t st);
template <typename TX, typename TY>
ctqr_status col_dot(int64_t rows, int S, const TX *x, int64_t ldx, const TY *y, int64_t ldy, double *out,
                    hipStream_t st);
template <typename TD, typename TS>
ctqr_status col_scale(int64_t rows, int S, const TS *src, int64_t lds, const double *dots, TD *dst, int64_t ldd,
                      hipStream_t st);
// x[r, s] /= sqrt(dots[s]) (row-major rows x S)
ctqr_status rm_scale(int64_t rows, int S, double *x, const double *dots, hipStream_t st);
ctqr_status cond_max(int S, const double *q, double *est, int slot, hipStream_t st);
ctqr_status cond_finish(const double *est, double *out, hipStream_t st);

// ---- tiles.hip (algorithm-by-blocks QR and solve) -------------------------------
#include <vector>
// task lists in the order of the paper's task tables (x type, y i, z k, w j)
std::vector<int4> tile_qr_tasks(int mt, int nt);
std::vector<int4> tile_solve_tasks(int mt, int nt);
// dependency level of each task (its reads and writes of blocks, S factors, B rows)
std::vector<int> tile_levels(const std::vector<int4> &tasks, int mt, int nt, bool solve);
// run the factorization / solve on the stream (dtasks: device room for the
// task list; waits on the stream once, after uploading it)
ctqr_status tile_qr_run(int m, int n, int b, double *A, int64_t lda, double *Sf, int4 *dtasks, hipStream_t st);
ctqr_status tile_solve_run(int m, int n, int b, const double *A, int64_t lda, const double *Sf, double *B,
                           int64_t ldb, int S, int4 *dtasks, hipStream_t st);


// ---- fused.hip (persistent solve kernels for few right-hand sides) -----------
constexpr int FUSED_MAX_S = 16;                   // slices the persistent kernels take
constexpr size_t FUSED_MAX_LDS = 150 * 1024;      // their LDS per workgroup, at most
int fused_grid();                                 // workgroups of a launch (compute units)
size_t fused_lds_bytes(int qmax, size_t esz);
// the rows of a right-hand side fit the launch's LDS
bool fused_fits(int64_t rows, size_t esz);
// elements of the exchange area (in the factor's precision), plus GB_WORDS
// barrier words
size_t fused_exchange_elems();
// R X = C (trans false) or R^T X = C (trans true) with the stored diagonal-block
// inverses; C is read only.  One cooperative launch; returns at once after
// the refinement's flag *skip is set.
template <typename T>
ctqr_status trsm_fused(int n, int S, bool trans, const T *R, int64_t ldr, const T *Rinv, const T *C, int64_t ldc,
                       T *X, int64_t ldx, T *ex, unsigned *bar, const int *skip, ctqr_info *info, hipStream_t st);
// Y = (Q^T B)[0:n] for FP64 B (m x S), in the factor's precision
template <typename T>
ctqr_status qtb_fused(int m, int n, int nb, int S, const T *QR, int64_t lda, const T *Tf, const double *B,
                      int64_t ldb, T *Y, int64_t ldy, T *ex, unsigned *bar, ctqr_info *info, hipStream_t st);
