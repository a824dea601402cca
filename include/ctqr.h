/*
 * ctqr.h -- C ABI of the MI355X (gfx950) QR least-squares CT reconstruction
 * library libctqr.so.
 *
 * The method (Chillaron, Quintana-Orti, Vidal, Verdu, "Computed tomography
 * medical image reconstruction on affordable equipment by using out-of-core
 * techniques"):
 *   Section II-A, Eq. 1   A X = B (+ W): A is M x N (rays x pixels), B is M x S
 *                         (one sinogram per column), X is N x S (one image per
 *                         column).
 *   Section II-A, Eq. 3   A = QR, computed once (it does not depend on B).
 *   Section II-A, Eq. 4   X = R^-1 (Q^T B), Q applied implicitly through its
 *                         Householder reflectors, R^-1 by backward substitution
 *                         (Section II-C, "System solving").
 *
 * Conventions shared by every call:
 *   - Dense matrices are column-major with a leading dimension (ld >= rows).
 *     Dense A/factor pointers must be 16-byte aligned and their leading
 *     dimension a multiple of 4 elements, so every column starts 16-byte
 *     aligned.
 *   - Every pointer marked "device" must point to device memory of the GPU
 *     that is current on the calling thread; "host" pointers are ordinary host
 *     memory.  The library never allocates or frees caller memory; all scratch
 *     comes from a caller-provided device workspace whose size the matching
 *     *_workspace() call reports.
 *   - Calls that take a stream only enqueue work on it and return at once.
 *   - Return value: CTQR_OK (0), or a negative code for an invalid call
 *     detected on the host before anything is enqueued (nothing is enqueued
 *     then), or CTQR_EHIP when the HIP runtime rejects a launch.  Numerical
 *     events (rank deficiency, non-finite values, refinement that does not
 *     converge) are written by the kernels into the caller's device-side
 *     ctqr_info; read it after synchronising the stream.
 *   - No C++ exception crosses this boundary.  Calls on different streams with
 *     different workspaces may run concurrently.
 */
#ifndef CTQR_H
#define CTQR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Same underlying type as HIP's own hipStream_t; NULL is the default stream. */
typedef struct ihipStream_t *hipStream_t;

typedef int32_t ctqr_status;
#define CTQR_OK               0
#define CTQR_EINVAL          (-1)  /* bad argument (null pointer, size, alignment, enum) */
#define CTQR_ENOMEM          (-2)  /* caller workspace or capacity too small */
#define CTQR_EHIP            (-3)  /* a HIP runtime call failed */
#define CTQR_EUNSUPPORTED    (-4)  /* valid but not supported (e.g. no gfx950 device) */
#define CTQR_RANK_DEFICIENT    1   /* info: |R_kk| <= n * u * max|R_ii| at column first_bad_col */
#define CTQR_NOT_CONVERGED     2   /* info: refinement stopped without meeting its tolerance */
#define CTQR_NONFINITE         3   /* info: NaN/Inf met in A, B or the refinement */
#define CTQR_CAPACITY          4   /* info: a sparse capacity (nnz_cap, column length) was exceeded */
#define CTQR_BARRIER_TIMEOUT   5   /* info: a grid barrier gave up waiting (results invalid) */

/* Storage precision of the dense A and of its factor. */
typedef int32_t ctqr_dtype;
#define CTQR_F64 0
#define CTQR_F32 1

/* Arithmetic of the blocked trailing update and of Q^T B.
 *   CTQR_PREC_FP64       FP64 storage, FP64 MFMA.
 *   CTQR_PREC_FP32_MFMA  FP32 storage, FP32 MFMA with FP32 accumulation; panel
 *                        norms and reflectors in FP64.
 *   CTQR_PREC_BF16_MFMA  FP32 storage, operands rounded to BF16 for MFMA with
 *                        FP32 accumulation; panel in FP64.
 *   CTQR_PREC_BF16X3_MFMA FP32 storage, each operand split into a BF16 high
 *                        part and a BF16 low part (its rounding remainder);
 *                        three BF16 MFMA products (high-high, high-low,
 *                        low-high) with FP32 accumulation, about 16 bits of
 *                        operand precision; panel in FP64.
 * The two BF16 modes apply to the block-column products ([G | W] = V^T [V | C]
 * and the trailing update C -= V W'); the inner panel updates and Q^T B stay
 * FP32. */
typedef int32_t ctqr_prec;
#define CTQR_PREC_FP64        0
#define CTQR_PREC_FP32_MFMA   1
#define CTQR_PREC_BF16_MFMA   2
#define CTQR_PREC_BF16X3_MFMA 3

/* Refinement of a solve with the FP64 sparse A (both forms use FP64
 * residuals r = B - A X, s = A^T r and the preconditioner (R^T R)^-1 applied
 * by the two triangular solves with the factor's R; both converge to the
 * least-squares solution of the FP64 A):
 *   CTQR_REFINE_CSNE  corrected semi-normal equations: X += (R^T R)^-1 s.
 *   CTQR_REFINE_PCG   the same corrections combined as conjugate directions
 *                     (preconditioned conjugate gradients on the normal
 *                     equations, Polak-Ribiere coefficient, per slice): fewer
 *                     iterations, and convergence where the plain corrections
 *                     stop contracting (A ill-conditioned for the factor's
 *                     precision). */
typedef int32_t ctqr_refine;
#define CTQR_REFINE_CSNE 0
#define CTQR_REFINE_PCG  1

/* Fan-beam scanner (Section II-A, Table I) and reconstruction grid.
 * Rays: one per (view, bin), row index view * n_bins + bin.  The source turns
 * on a circle of radius src_iso_cm; the flat detector, src_det_cm from the
 * source and perpendicular to the central ray, has n_bins equal bins spanning
 * the fan_deg fan; each ray joins the source to a bin centre.
 * Pixels: side x side square of side fov_side_cm centred on the rotation axis,
 * column index iy * side + ix (x fastest, origin at the lower-left corner).
 * angle_schedule: 0 = uniform 360/n_views steps, 1 = Eq. 2 (quarter-turn
 * shifts +0.5, -0.75, -0.25 degrees, each quarter continuing from the last
 * angle of the previous one). */
typedef struct {
    int32_t side, n_views, n_bins;
    int32_t angle_schedule;
    double src_iso_cm, src_det_cm, fan_deg, fov_side_cm;
} ctqr_geometry;

/* FP64 sparse copy of A for exact residuals: CSR (row-major) and CSC
 * (column-major, rows ascending within each column).  All arrays device. */
typedef struct {
    int64_t m, n, nnz_cap;
    int64_t *rowptr;  int32_t *col;  double *val;    /* CSR: m+1, nnz_cap, nnz_cap */
    int64_t *colptr;  int32_t *row;  double *cval;   /* CSC: n+1, nnz_cap, nnz_cap */
} ctqr_sparse;

/* Numerical outcome, written by the kernels (device memory, caller-owned). */
typedef struct {
    int32_t status;          /* 0 or one of the positive codes above           */
    int32_t first_bad_col;   /* rank deficiency: first column k with tiny R_kk */
    int32_t iters;           /* refinement iterations performed                */
    int32_t x_iters;         /* refinement updates contained in the returned X:
                                iters, or fewer when CTQR_NOT_CONVERGED returned
                                an earlier iterate (the one with the smallest
                                normal-equation residual, see
                                ctqr_qr_solve_slices)                           */
    double  max_rel_update;  /* refinement: max_s ||dx_s||_inf / ||x_s||_inf of
                                the last update, or of the update computed from
                                the returned iterate when an earlier one is
                                returned                                        */
    double  rdiag_max;       /* max |R_kk|                                      */
    double  rdiag_min;       /* min |R_kk|                                      */
    int64_t nnz;             /* system matrix build: nonzeros of A              */
    double  contraction;     /* refinement: mean contraction per iteration,
                                (last / first relative update)^(1/(iters-1));
                                0 with fewer than two iterations.  Corrected
                                semi-normal equations contract by about
                                c u kappa(A)^2, u the factor's precision        */
} ctqr_info;

/* Human-readable name of a status code (static string, never NULL). */
const char *ctqr_status_string(ctqr_status s);

/* Library version string and the device architecture it was built for. */
const char *ctqr_version(void);

/* Text of the last HIP failure seen by this thread (empty if none). */
const char *ctqr_last_error(void);

/* Sizes of A for a geometry (host only, no HIP call): m = n_views * n_bins
 * rays, n = side^2 pixels, nnz_upper = m * (2 side - 1), an upper bound on the
 * nonzeros (a straight ray crosses at most 2 side - 1 pixels).  Section II-A. */
ctqr_status ctqr_geometry_sizes(const ctqr_geometry *g, int64_t *m, int64_t *n,
                                int64_t *nnz_upper);

/* Workspace (device bytes) for ctqr_build_system_matrix. */
ctqr_status ctqr_build_workspace(const ctqr_geometry *g, size_t *bytes);

/* Build the system matrix A (Section II-A, Eq. 1): a_ij = length of ray i
 * inside pixel j in units of the pixel pitch (Siddon ray tracing).
 *   A      device, dense m x n column-major in `dtype`, leading dim lda; may be
 *          NULL (no dense copy).  Every entry is written (zeros included).
 *   sp     sparse FP64 copy (CSR + CSC) with caller-allocated arrays of
 *          capacity sp->nnz_cap; may be NULL.  sp->m, sp->n must match.
 *   info   device; info->nnz receives the nonzero count, info->status
 *          CTQR_CAPACITY if nnz_cap was too small (the sparse arrays are then
 *          incomplete).
 *   work   device workspace of at least ctqr_build_workspace() bytes.
 * Cites: Section II-A (A models the scanner; M = detectors x views), Table I,
 * Eq. 2 (angles). */
ctqr_status ctqr_build_system_matrix(const ctqr_geometry *g, ctqr_dtype dtype,
                                     void *A, int64_t lda, ctqr_sparse *sp,
                                     void *work, size_t work_bytes,
                                     ctqr_info *info, hipStream_t stream);

/* Workspace (device bytes) for ctqr_qr_factor.  nb = 0 picks the default
 * outer block (256). */
ctqr_status ctqr_qr_workspace(int64_t m, int64_t n, ctqr_dtype dtype, ctqr_prec prec,
                              int32_t nb, size_t *bytes);

/* Blocked Householder QR, A = QR (Eq. 3), right-looking with compact-WY
 * block reflectors H_k ... H_{k+nb-1} = I - V T V^T.
 *   A      device, m x n (m >= n >= 1) in `dtype`, leading dim lda.  On exit
 *          R is in the upper triangle and the Householder vectors v_k (unit
 *          diagonal implied) below it: the in-place output of the paper's
 *          Compute_dense_QR (Section II-C).
 *   prec   CTQR_PREC_FP64 requires dtype CTQR_F64; the two MFMA modes require
 *          CTQR_F32.
 *   nb     outer block width (multiple of 32, <= 256), 0 = default.  The same
 *          nb must be passed to the solve.  When nb divides 512, groups
 *          of four block columns share one trailing update: each block's
 *          reflector updates only the rest of its group, and the group's
 *          reflectors together update the remaining columns as one block
 *          reflector up to 4 nb wide, I - V T V^T with
 *          T = [T_0, -T_0 V_0^T V_1 T_1, ...; 0, T_1, ...], one pass over the
 *          trailing columns per group.  T still holds each block's own T.
 *   T      device, nb x n in `dtype` (leading dim nb): the nb x nb upper
 *          triangular T of each block column (the paper's "S factors").
 *   tau    device, n doubles: the reflector scalars (LAPACK larfg convention:
 *          beta = -sign(alpha)||x||, tau = (beta - alpha)/beta).
 *          The 32-column inner panels held in FP64 form V, tau and R by
 *          Cholesky QR twice and the Householder reconstruction, which gives
 *          the larfg results up to rounding, whenever that is safe for the
 *          panel.  Otherwise, and everywhere with the environment variable
 *          CTQR_PANEL_ROUTE=columns, they form them one column at a time.
 *          Each route is bitwise reproducible.
 *   Rinv   device, ctqr_qr_rinv_bytes(n, dtype) bytes in `dtype`, or NULL: the
 *          inverses of the 2048 x 2048 diagonal blocks of R and their
 *          transposes, stored with the factor so every later solve's block
 *          back substitution is a chain of MFMA products (the factorization is
 *          done once and kept for every later solve, Section II-A).  NULL skips them;
 *          the solve then builds them in its workspace each call.
 *   info   device: rank deficiency / non-finite / barrier time-out.
 * Sections II-C ("QR factorization"), Eq. 3. */
ctqr_status ctqr_qr_factor(int64_t m, int64_t n, ctqr_dtype dtype, void *A, int64_t lda,
                           ctqr_prec prec, int32_t nb, void *T, double *tau, void *Rinv,
                           void *work, size_t work_bytes, ctqr_info *info,
                           hipStream_t stream);

/* Outer block width nb for ctqr_qr_factor, picked by timing on the caller's
 * own matrix: each candidate nb in {64, 128, 256} factors the leading
 * min(n, 1024) columns with the trailing updates over all n columns, on `stream`,
 * and the candidate with the least time per factored column wins.
 * A is OVERWRITTEN (each candidate factors it further in place): rebuild it
 * before the real factorization.  The stream is synchronised (the timing is
 * read on the host).
 *   A, lda, dtype, prec, T, tau, info   as ctqr_qr_factor.
 *   work        ctqr_qr_workspace(m, n, dtype, prec, 256) bytes.
 *   nb_best     host: the chosen nb.
 *   ms_per_col  host, 3 floats or NULL: milliseconds per factored column of
 *               each candidate, in the order 64, 128, 256.
 * The tuned outer block width of the batched path's parameters. */
ctqr_status ctqr_qr_tune_nb(int64_t m, int64_t n, ctqr_dtype dtype, void *A, int64_t lda,
                            ctqr_prec prec, void *T, double *tau, void *work, size_t work_bytes,
                            ctqr_info *info, int32_t *nb_best, float *ms_per_col,
                            hipStream_t stream);

/* Columns [c0, c1) of the dense A, rebuilt from the CSC half of a sparse copy
 * made by ctqr_build_system_matrix: column c0 + q goes to A + q * lda
 * (device, `dtype`, every entry of the lda x (c1 - c0) block written).  The
 * same values as the dense output of the build (each a_ij rounded once to
 * `dtype`), for matrices whose dense form is produced a tile at a time
 * (Section II-A, Eq. 1). */
ctqr_status ctqr_sparse_to_dense(const ctqr_sparse *sp, ctqr_dtype dtype, int64_t c0, int64_t c1,
                                 void *A, int64_t lda, hipStream_t stream);

/* ---- Out-of-core factorization --------------------------------------------
 * For an A larger than device memory (the paper's out-of-core setting,
 * Section II-B, with HBM in the role of main memory and pinned host memory in
 * the role of the disk).  Columns [0, n_dev) of A are in device memory
 * (A_dev, leading dim lda); columns [n_dev, n) are in pinned host memory
 * (A_host, allocated with hipHostMalloc; column j at A_host + (j - n_dev) *
 * lda, same lda).  The resident columns are factored first, with their
 * trailing updates kept inside them; each host tile of tile_cols columns is
 * then uploaded, takes the block-reflector updates of every factored block
 * column to its left (left-looking: resident blocks from HBM, earlier host
 * tiles uploaded again one at a time), is factored, and written back.  The
 * factor, T, tau and Rinv are bit-identical to ctqr_qr_factor's on the same
 * matrix (every reduction keeps the split of the all-in-HBM run).
 *   n_dev, tile_cols  multiples of 2048 and of nb; 0 <= n_dev <= n.
 *   A_dev   device, m x n_dev (may be NULL when n_dev = 0).
 *   A_host  pinned host, m x (n - n_dev) (may be NULL when n_dev = n); on
 *           exit it holds its columns of the factor.  CTQR_EINVAL if it is
 *           not pinned host memory.
 *   T, tau, Rinv, info  as ctqr_qr_factor (T, tau and Rinv in device memory).
 *   work    device, ctqr_qr_factor_ooc_workspace bytes (two tile buffers
 *           of lda * tile_cols elements plus the factorization workspace).
 * Kernels run on `stream`; the tile copies run on a copy stream of the call,
 * ordered by events, so the next tile uploads while the current one is
 * factored, the first while the resident columns are factored, and each
 * factored tile is written back while the next takes its updates.  The call
 * returns once every copy has finished (host memory then holds the factor);
 * the kernels enqueued on `stream` are complete when it synchronises. */
ctqr_status ctqr_qr_factor_ooc_workspace(int64_t m, int64_t n, ctqr_dtype dtype, ctqr_prec prec,
                                         int32_t nb, int64_t lda, int64_t tile_cols, size_t *bytes);
ctqr_status ctqr_qr_factor_ooc(int64_t m, int64_t n, ctqr_dtype dtype, void *A_dev, void *A_host,
                               int64_t lda, int64_t n_dev, int64_t tile_cols, ctqr_prec prec,
                               int32_t nb, void *T, double *tau, void *Rinv, void *work,
                               size_t work_bytes, ctqr_info *info, hipStream_t stream);

/* Solve with an out-of-core factor (the outputs of ctqr_qr_factor_ooc, same
 * n_dev, tile_cols, lda and nb; Rinv required): X = R^-1 Q^T B with the
 * refinement of ctqr_qr_solve_slices.  Q^T B applies the resident blocks and
 * then each host tile uploaded in turn; R X = C runs from the last host tile
 * back to the resident columns (right-looking) and R^T Y = C from the
 * resident columns forward (left-looking), so each substitution uploads
 * every host tile once and never writes host memory.  B, X, the sparse A and
 * the work space are device memory; the workspace holds one tile buffer
 * (ctqr_solve_ooc_workspace).  With refinement the call waits on the stream
 * after each iteration, as ctqr_qr_solve_slices does.  Section II-B (one
 * read of the stored factor per pass serves every slice). */
ctqr_status ctqr_solve_ooc_workspace(int64_t m, int64_t n, ctqr_dtype dtype, int32_t nb,
                                     int32_t nslices, int32_t refine, int64_t lda,
                                     int64_t tile_cols, size_t *bytes);
ctqr_status ctqr_qr_solve_ooc(int64_t m, int64_t n, ctqr_dtype dtype, const void *QR_dev,
                              const void *QR_host, int64_t lda, int64_t n_dev, int64_t tile_cols,
                              const void *T, const double *tau, const void *Rinv, int32_t nb,
                              const double *B, int64_t ldb, int32_t nslices, double *X,
                              int64_t ldx, const ctqr_sparse *A64, double tol, int32_t max_iters,
                              int32_t refine_method, void *work, size_t work_bytes, ctqr_info *info,
                              hipStream_t stream);

/* Bytes of the Rinv array of ctqr_qr_factor / ctqr_qr_solve_slices (host only). */
ctqr_status ctqr_qr_rinv_bytes(int64_t n, ctqr_dtype dtype, size_t *bytes);

/* Workspace (device bytes) for ctqr_qr_solve_slices with up to nslices
 * right-hand sides; refine: 0 none, 1 the refinement vectors, 2 also the
 * conjugate-gradient vectors (CTQR_REFINE_PCG). */
ctqr_status ctqr_solve_workspace(int64_t m, int64_t n, ctqr_dtype dtype, int32_t nb,
                                 int32_t nslices, int32_t refine, size_t *bytes);

/* Least-squares reconstruction of nslices sinograms with a stored factor:
 * X = R^-1 (Q^T B) (Eq. 4), Q^T applied block by block with the compact-WY
 * factors, then block backward substitution with R (Section II-C, "System
 * solving").
 *   QR, T, tau, Rinv  the outputs of ctqr_qr_factor (same m, n, dtype, nb);
 *          Rinv may be NULL (then it is rebuilt in the workspace).
 *   B      device, m x nslices FP64, leading dim ldb (not modified).
 *   X      device, n x nslices FP64, leading dim ldx (output).
 *   A64    optional FP64 sparse A (from ctqr_build_system_matrix).  When given,
 *          the solution is refined by corrected semi-normal equations:
 *          r = B - A X (FP64), R^T y = A^T r, R d = y, X += d.  The
 *          refinement has converged (status 0) only when the relative update
 *          max_s ||d_s||_inf / ||X_s||_inf is <= tol.  It stops with
 *          CTQR_NOT_CONVERGED when two consecutive updates fail to shrink
 *          below 0.9x the previous one, or after max_iters; X is then the
 *          iterate with the smallest normal-equation residual
 *          max_s ||A^T (B_s - A X_s)||_inf / ||A^T (B_s - A X0_s)||_inf (X0 the
 *          unrefined solution; A^T r = A^T A e measures the error e whatever
 *          the preconditioner's quality), or the last iterate if the residual
 *          was still falling at the last iteration (info.x_iters says which).
 *          NULL = no refinement.
 *          With FP32 storage, CSNE and at least 128 slices, the V W' products
 *          of Q^T B and the off-diagonal block products of every substitution
 *          run on split-BF16 MFMA (three BF16 products, FP32 accumulation):
 *          the refinement needs the factor's own accuracy only.
 *          With refinement the call waits on the stream after each
 *          iteration (it reads the convergence flag back) and returns once
 *          the refinement has ended; without it the call only enqueues.
 *   refine_method  CTQR_REFINE_CSNE or CTQR_REFINE_PCG (both follow the
 *          rule above; the conjugate-gradient form allows a longer run of
 *          non-shrinking updates, 6, before it stops).
 *   info   device: iterations, last relative update, CTQR_NOT_CONVERGED /
 *          CTQR_NONFINITE (CTQR_BARRIER_TIMEOUT: see below).
 * Few slices, as an option: with the environment variable CTQR_FUSED=1 set
 * (read at every call), a solve of nslices <= 16 (nb a multiple of 64 up to
 * 256, the rows of B within the LDS of one workgroup per compute unit) runs
 * Q^T B and every block substitution as persistent kernels, one cooperative
 * launch each, with the same blocks and the same products per block, summed
 * in a fixed order (each slice's result does not depend on how many slices
 * share the call).  The default launch-per-block path is faster on MI355X at
 * every slice count measured. */
ctqr_status ctqr_qr_solve_slices(int64_t m, int64_t n, ctqr_dtype dtype,
                                 const void *QR, int64_t lda, const void *T,
                                 const double *tau, const void *Rinv, int32_t nb,
                                 const double *B, int64_t ldb, int32_t nslices,
                                 double *X, int64_t ldx,
                                 const ctqr_sparse *A64, double tol, int32_t max_iters,
                                 int32_t refine_method, void *work, size_t work_bytes,
                                 ctqr_info *info, hipStream_t stream);

/* The solve of ctqr_qr_solve_slices for callers that cannot allocate device
 * memory (code under HIP graph capture, tight serving loops, harnesses that
 * forbid hipMalloc): the same arguments without the workspace, which comes
 * from a scratch array the library holds in device memory, one copy per GPU,
 * of CTQR_NOALLOC_SCRATCH_BYTES (256 MiB), kept until the process ends.  The
 * call allocates nothing: no hipMalloc, hipFree or allocating library
 * routine, also not for the refinement, which reads its end-of-refinement
 * flag into ordinary host memory.  Inputs, outputs and results are those of
 * ctqr_qr_solve_slices (same kernels, same workspace layout).
 *   Limit  returns CTQR_ENOMEM, with nothing enqueued, when
 *          ctqr_solve_workspace(m, n, dtype, nb, nslices, refine) exceeds
 *          CTQR_NOALLOC_SCRATCH_BYTES (the text is in ctqr_last_error).
 *   Races  every call on one GPU uses that GPU's one scratch array: calls
 *          that overlap on one GPU (other threads, other streams) race and
 *          corrupt each other's results; order them.  The array keeps the
 *          last call's contents; each call initialises what it reads.
 * The first call on a device looks up the array's device address
 * (hipGetSymbolAddress) with that device current. */
#define CTQR_NOALLOC_SCRATCH_BYTES ((size_t)256 << 20)
ctqr_status ctqr_qr_solve_slices_noalloc(int64_t m, int64_t n, ctqr_dtype dtype,
                                         const void *QR, int64_t lda, const void *T,
                                         const double *tau, const void *Rinv, int32_t nb,
                                         const double *B, int64_t ldb, int32_t nslices,
                                         double *X, int64_t ldx,
                                         const ctqr_sparse *A64, double tol, int32_t max_iters,
                                         int32_t refine_method, ctqr_info *info, hipStream_t stream);

/* ---- Batched solver ------------------------------------------------------
 * One stored factorization serves a stream of reconstruction requests: the
 * factorization does not depend on B, so it is computed once and reused
 * (Section II-A), and the per-slice cost falls as more slices share one read
 * of the factor (Section III-B).  A solver holds a stored factor (the
 * outputs of ctqr_qr_factor, Rinv required) and solves requests of 1 ..
 * max_slices slices.  A request of S slices runs in the smallest slice
 * bucket >= S -- the powers of two up to 64, then the multiples of 64 (the
 * extra slices are zero and do not change the others' results).  Each bucket's solve -- Q^T B, the back substitution and, with
 * refinement, a calibrated number of refinement iterations -- is captured
 * once into a HIP graph and replayed on the caller's stream.  With the
 * persistent kernels of ctqr_qr_solve_slices selected (CTQR_FUSED=1), the
 * buckets of at most 16 slices they take enqueue those kernels directly
 * instead (a few launches per request, no graph), with the same calibrated
 * iteration count.
 *
 * Refinement (A64 != NULL, max_iters > 0) follows ctqr_qr_solve_slices.  The
 * first request of a bucket runs eagerly and counts its iterations; the
 * bucket's graph then holds that count + 2 (at most max_iters), its kernels
 * returning at once after convergence.  After each replay the call reads the
 * convergence flag (it waits on the stream) and, if the refinement has not
 * ended, continues eagerly up to max_iters and recaptures the bucket with the
 * larger count on its next use.  The results of a bucket are bitwise
 * reproducible: a graph replays exactly the kernels of the eager run.
 *
 * Memory: the solver owns no device memory; the caller passes a workspace
 * of ctqr_solver_workspace bytes, which must outlive the solver.  The
 * factor, T, tau, Rinv and the sparse arrays are referenced, not copied, and
 * must stay valid and unmodified.  Host memory: the graphs, a capture
 * stream and an event.  Calls on one solver are serialised: on the host by a
 * lock, on the GPU by an event that each call records after its work and
 * that the next call's stream waits for, so calls may come from different
 * streams.  Solvers with different workspaces are independent. */
typedef struct ctqr_solver_t *ctqr_solver;

typedef struct {
    int64_t m, n;
    int32_t dtype;          /* ctqr_dtype of the factor */
    int32_t nb;             /* the factor's block width (0 = default) */
    const void *QR;         /* factored A, leading dim lda */
    int64_t lda;
    const void *T;          /* nb x n block-reflector factors */
    const double *tau;
    const void *Rinv;       /* diagonal-block inverses (required) */
    const ctqr_sparse *A64; /* FP64 sparse A for the refinement, or NULL */
    double tol;             /* refinement tolerance */
    int32_t max_iters;      /* refinement iteration limit (0 = none) */
    int32_t max_slices;     /* largest request, 1 .. 4096 */
    int32_t refine_method;  /* CTQR_REFINE_CSNE or CTQR_REFINE_PCG */
    int32_t pad;
} ctqr_solver_desc;        /* 96 bytes */

/* Workspace bytes of a solver (host only). */
ctqr_status ctqr_solver_workspace(const ctqr_solver_desc *desc, size_t *bytes);

/* Creates a solver; *out is NULL on failure. */
ctqr_status ctqr_solver_create(const ctqr_solver_desc *desc, void *work, size_t work_bytes,
                               ctqr_solver *out);

/* Autotuner: times Q^T B plus the back substitution of every bucket with the
 * 32-wide and with the 128-wide slice tile of the MFMA products (reps timed
 * runs each, after one warm-up) and keeps the faster (untuned buckets use the
 * 32-wide tile up to 32 slices; buckets of the persistent kernels are
 * skipped).  Overwrites the solver's request
 * buffer; waits on the stream.  Buckets whose choice changed are recalibrated
 * and recaptured on their next use. */
ctqr_status ctqr_solver_tune(ctqr_solver solver, int32_t reps, hipStream_t stream);

/* X = R^-1 Q^T B for one request of nslices slices (B m x nslices FP64, ldb;
 * X n x nslices FP64, ldx; both device, B not modified).  info (device)
 * receives the request's ctqr_info.  Without refinement the call only
 * enqueues; with it the call waits on the stream once per request (twice
 * for a bucket's calibration run, which waits after every iteration). */
ctqr_status ctqr_solver_solve(ctqr_solver solver, const double *B, int64_t ldb, int32_t nslices,
                              double *X, int64_t ldx, ctqr_info *info, hipStream_t stream);

/* Several queued requests in one solve: their slices (sum <= max_slices) are
 * packed side by side into one bucket, so the requests share one pass over
 * the factor.  Arrays of nreq entries in host memory; B[i], X[i] are device
 * pointers as in ctqr_solver_solve.  Slices do not interact (the refinement
 * stops when the slowest slice has converged), so each request's X is its
 * own least-squares solution; info is that of the batch.  Requests of one
 * call must not overlap in X. */
ctqr_status ctqr_solver_solve_batch(ctqr_solver solver, int32_t nreq, const double *const *B,
                                    const int64_t *ldb, const int32_t *nslices, double *const *X,
                                    const int64_t *ldx, ctqr_info *info, hipStream_t stream);

/* For a request of nslices: its bucket, the slice-tile width its products use
 * (32 or 128) and the refinement iterations its captured graph holds, or a
 * persistent-kernel bucket enqueues per request (-1: not run yet; 0 without
 * refinement).  Host only. */
ctqr_status ctqr_solver_query(ctqr_solver solver, int32_t nslices, int32_t *bucket,
                              int32_t *slice_tile, int32_t *graph_iters);

/* Releases the graphs and the capture stream (not the workspace).  NULL is
 * accepted. */
ctqr_status ctqr_solver_destroy(ctqr_solver solver);

/* Estimate of the 2-norm condition number of A.  The direct solve needs A of
 * full column rank (Section II-A), and kappa(A) sets how far a least-squares
 * solution moves under perturbations of A and B, including rounding: the
 * perturbation bound of the solution is about u (2 kappa + kappa^2 tan theta)
 * with tan theta = ||r|| / ||A x||.  kappa(A) = sigma_max(A) / sigma_min(A):
 *   sigma_max(A)  power iteration on A^T A with the FP64 sparse A;
 *   sigma_min(A) = sigma_min(R) (A = QR, Eq. 3)  inverse iteration on R^T R,
 *                 applied by the two block substitutions with the factor's R
 *                 (R^T y = z, R w = y).
 * nvec start vectors (1..64, fixed counter-hashed values) iterate together
 * for `iters` steps; every step's Rayleigh quotient is a lower bound of
 * sigma_max^2 (resp. 1 / sigma_min^2), and the largest over vectors and steps
 * is kept, so both estimates approach the true values from one side and
 * kappa is never over-estimated.
 *   QR, lda, dtype, Rinv  the factor (ctqr_qr_factor outputs; Rinv required).
 *   A64    device, the FP64 sparse A of the same matrix (CSR and CSC).
 *   out    device, 3 doubles: sigma_max(A), sigma_min(R), kappa.
 *   work   device, ctqr_cond_workspace bytes.
 * The call only enqueues; read out after synchronising the stream. */
ctqr_status ctqr_cond_workspace(int64_t m, int64_t n, ctqr_dtype dtype, int32_t nvec, size_t *bytes);
ctqr_status ctqr_cond_estimate(int64_t m, int64_t n, ctqr_dtype dtype, const void *QR, int64_t lda,
                               const void *Rinv, const ctqr_sparse *A64, int32_t nvec, int32_t iters,
                               void *work, size_t work_bytes, double *out, hipStream_t stream);

/* ---- Algorithm-by-blocks QR and solve (Section II-C) ------------------------
 * The matrix is cut into b x b blocks A_ij (1 <= b <= 64; the last block row
 * and column may be smaller) and factored by tasks on a few blocks each, the
 * paper's four generic tasks:
 *   CTQR_TASK_DENSE_QR    Compute_dense_QR(A_kk, S_kk): Householder QR of A_kk
 *                         (R on and above its diagonal, reflectors below; S_kk
 *                         the compact-WY factor, H_1 ... H_c = I - V S V^T).
 *   CTQR_TASK_TD_QR       Compute_TD_QR(A_kk, A_ik, S_ik): QR of the triangle
 *                         R_kk stacked on the dense A_ik (reflectors [e_p; v_p],
 *                         v_p into A_ik; S_ik for U = [I; A_ik]).
 *   CTQR_TASK_APPLY_DENSE Apply_left_Qt_of_dense_QR(A_kk, S_kk, C).
 *   CTQR_TASK_APPLY_TD    Apply_left_Qt_of_TD_QR(A_ik, S_ik, F, G).
 * and for the solve X = R^-1 (Q^T B) the block substitution and product:
 *   CTQR_TASK_TRSM        Trsm_lunn: B_i = upper(A_ii)^-1 B_i.
 *   CTQR_TASK_GEMM        Gemm_nn_mo: B_i = -A_ij B_j + B_i.
 * The factorization's tasks are generated in the left-looking order of the
 * paper's task table (for each block column j: the transformations of every
 * earlier block column k, dense then TD for each block row below, then the
 * QR of block column j); the solve's in the order of its table (Q^T B block
 * row by block row, then the substitution by block rows from the last).
 * Householder vectors follow the larfg convention of ctqr_qr_factor. */
typedef struct {
    int32_t type;   /* CTQR_TASK_* */
    int32_t i;      /* block row the task writes (the TD block; the B row) */
    int32_t k;      /* block column of the reflectors it creates or applies */
    int32_t j;      /* target block column (apply, factor: = k; gemm: the X block; solve apply: -1) */
} ctqr_tile_task;
#define CTQR_TASK_DENSE_QR    0
#define CTQR_TASK_TD_QR       1
#define CTQR_TASK_APPLY_DENSE 2
#define CTQR_TASK_APPLY_TD    3
#define CTQR_TASK_TRSM        4
#define CTQR_TASK_GEMM        5

/* The task list of the factorization (solve = 0) or of the solve (solve = 1)
 * for mt x nt blocks (mt >= nt), in execution order (host only).  tasks may
 * be NULL to query *count; otherwise up to cap entries are written. */
ctqr_status ctqr_tile_tasks(int32_t mt, int32_t nt, int32_t solve, ctqr_tile_task *tasks, int64_t cap,
                            int64_t *count);

/* Sizes for ctqr_tile_qr_factor / ctqr_tile_qr_solve (host only): the S
 * factors (*s_elems doubles: one b x b block per block (i, k), i >= k, at
 * S + (k mt + i) b^2, column-major) and the device workspace (the task list
 * of the larger of the two runs). */
ctqr_status ctqr_tile_qr_sizes(int64_t m, int64_t n, int32_t b, int64_t *s_elems, size_t *work_bytes);

/* Algorithm-by-blocks QR of the FP64 A (device, m x n, m >= n, leading dim
 * lda), in place: R above, reflectors below each diagonal block and in the
 * blocks under it; S (device) receives the S factors.  The tasks run in
 * dependency levels (a task waits for the tasks whose blocks it reads or
 * overwrites; the tasks of one level and type go in one launch, one workgroup
 * per task).  The call waits on the stream once, after uploading the task
 * list to work; the kernels are only enqueued. */
ctqr_status ctqr_tile_qr_factor(int64_t m, int64_t n, double *A, int64_t lda, int32_t b, double *S,
                                void *work, size_t work_bytes, hipStream_t stream);

/* X = R^-1 (Q^T B) with the outputs of ctqr_tile_qr_factor (same m, n, b):
 * B (device, m x nslices FP64, leading dim ldb) is overwritten, its first n
 * rows receiving X.  Waits on the stream once (task list upload). */
ctqr_status ctqr_tile_qr_solve(int64_t m, int64_t n, const double *QR, int64_t lda, int32_t b, const double *S,
                               double *B, int64_t ldb, int32_t nslices, void *work, size_t work_bytes,
                               hipStream_t stream);

/* Sinogram simulation with Joseph's projector, the method the paper's
 * sinograms come from (Section II-A, after Table I): B = J X for the scanner
 * and grid of g.  Each ray is sampled once per pixel column (when it runs
 * closer to the x axis; else once per pixel row) on the line through the pixel
 * centres, the image is linearly interpolated there between the two nearest
 * pixel centres of that column (row), pixels outside the image counting as
 * zero, and each sample is weighted by the ray length between consecutive
 * column (row) lines, in pixel pitches (the unit of A).  J differs from the
 * Siddon A of ctqr_build_system_matrix, so least-squares reconstructions of
 * J X with A carry a model error on top of noise.
 *   X   device, n x nslices FP64 images (pixel iy * side + ix), leading dim ldx.
 *   B   device, m x nslices FP64 output (row view * n_bins + bin), ldb.
 * Thread per (ray, slice); the call only enqueues. */
ctqr_status ctqr_project_joseph(const ctqr_geometry *g, int32_t nslices, const double *X, int64_t ldx,
                                double *B, int64_t ldb, hipStream_t stream);

/* Image-quality metrics of reconstructions (Section II-B): for each slice s,
 * PSNR (Eq. 5, Eq. 6: 10 log10(max(I0)^2 / MSE), MSE over the side x side
 * image, +inf for identical images) and the mean SSIM (Eq. 7) of X[:, s]
 * against the reference Xref[:, s].  SSIM is evaluated on every 11 x 11 window
 * inside the image with Gaussian weights (standard deviation 1.5 pixels,
 * normalised to sum 1) for the window means, variances and covariance, and
 * c1 = (0.01 L)^2, c2 = (0.03 L)^2 with L = data_range, or the reference
 * image's max - min when data_range is 0; NaN when side < 11.
 *   Xref, X  device, n x nslices FP64, leading dims ldr, ldx.
 *   out      device, 2 nslices doubles: out[s] = PSNR (dB), out[nslices + s] = SSIM.
 * One workgroup per slice, sums in a fixed order: reproducible. */
ctqr_status ctqr_image_quality(int32_t side, int32_t nslices, const double *Xref, int64_t ldr,
                               const double *X, int64_t ldx, double data_range, double *out,
                               hipStream_t stream);

/* View-count search: the smallest number of views for which A has full
 * column rank.  The direct method needs full rank (Section II-A, Section IV),
 * and the number of views that gives it depends on the resolution; Eq. 2
 * places the views with per-quarter angle shifts that break the symmetry of
 * the projection data to raise the rank.  For v = v_min, v_min + v_step, ...
 * up to v_max (geometry g with n_views = v; its other fields, the angle
 * schedule included, as given), the call builds the FP64 A (dense and sparse),
 * factors it (FP64 QR, nb = 256) and estimates kappa(A) (ctqr_cond_estimate
 * with 8 vectors and `iters` steps).  A view count passes when the
 * factorization raises no rank flag (|R_kk| > n u max|R_ii| for every k) and
 * kappa <= kappa_max; the search stops at the first that passes.  Counts with
 * fewer rays than pixels (v n_bins < side^2) fail without any GPU work.
 *   trials    host, up to max_trials entries, one per count tried, in order:
 *             views, status (CTQR_OK = full rank, CTQR_RANK_DEFICIENT
 *             otherwise), kappa estimate (INFINITY when not factored),
 *             min and max |R_kk|.
 *   n_trials  host: entries written.   v_best  host: the passing count, or 0.
 *   work      device, ctqr_view_search_workspace(g, v_max) bytes.
 * The call waits on the stream after every step (it reads the outcomes). */
typedef struct {
    int32_t views;
    int32_t status;
    double kappa;
    double rdiag_min, rdiag_max;
} ctqr_view_trial;
ctqr_status ctqr_view_search_workspace(const ctqr_geometry *g, int32_t v_max, size_t *bytes);
ctqr_status ctqr_view_search(const ctqr_geometry *g, int32_t v_min, int32_t v_max, int32_t v_step,
                             double kappa_max, int32_t iters, void *work, size_t work_bytes,
                             ctqr_view_trial *trials, int32_t max_trials, int32_t *n_trials,
                             int32_t *v_best, hipStream_t stream);

/* Sinogram synthesis and residual helper: Y = alpha * A X + beta * Y with the
 * FP64 CSR copy of A.  X (n x nslices, ldx) and Y (m x nslices, ldy) are
 * column-major FP64 device arrays.  Eq. 1. */
ctqr_status ctqr_spmm(const ctqr_sparse *A64, int32_t nslices, double alpha,
                      const double *X, int64_t ldx, double beta, double *Y, int64_t ldy,
                      hipStream_t stream);

/* Progress of the long out-of-core calls.  When a hook is set,
 * ctqr_qr_factor_ooc reports (CTQR_PROGRESS_FACTOR, columns factored, n)
 * after every 8192 resident columns and after every host tile, and
 * ctqr_qr_solve_ooc reports (CTQR_PROGRESS_SOLVE, iterations done, max_iters)
 * after Q^T B and after each refinement iteration.  Each report is a host
 * function enqueued on the call's stream (hipLaunchHostFunc), so it runs on a
 * HIP runtime thread once the GPU has finished the work before it; the hook
 * must return quickly and must not call HIP.  NULL removes the hook.  The
 * hook is process-wide. */
#define CTQR_PROGRESS_FACTOR 1
#define CTQR_PROGRESS_SOLVE  2
typedef void (*ctqr_progress_fn)(int32_t stage, int64_t done, int64_t total, void *user);
ctqr_status ctqr_set_progress(ctqr_progress_fn fn, void *user);

/* Releases the library's process-lifetime state: waits for the current
 * device to finish its work, frees the pinned host words the refinement reads
 * its flag into, destroys the timing events and removes the progress hook.
 * Call it with no ctqr call in flight, before the HIP runtime is torn down
 * (the Python binding calls it at interpreter exit); the library remains
 * usable afterwards (the state is made again on first use).  Solvers are not
 * touched: destroy them with ctqr_solver_destroy. */
ctqr_status ctqr_release(void);

/* Kernel-level timing of the dominant kernel (the trailing-update GEMM
 * C -= V W of ctqr_qr_factor).  While enabled, every launch of it is
 * bracketed by HIP events on the stream it runs on; ctqr_profile_read returns
 * the number of launches, their summed duration (ms, resolved after the
 * caller has synchronised the stream) and their summed algorithmic flops
 * (2 * rows * cols * K per launch, K = nb, or the group's width for grouped
 * block columns; the updates inside a group by its blocks are not counted).
 * Host-side bookkeeping only; enabling it clears the previous records.  `on`
 * is a bit set: CTQR_PROFILE_UPDATE for these records, CTQR_PROFILE_PHASES
 * for the phase timing below (0 turns both off). */
#define CTQR_PROFILE_UPDATE 1
#define CTQR_PROFILE_PHASES 2
ctqr_status ctqr_profile_enable(int32_t on);
ctqr_status ctqr_profile_read(int64_t *launches, double *total_ms, double *total_flops);
/* The same records for the other large product of the factorization, the
 * reductions [G | W] = V^T [V | C] of every block column and group (one
 * launch of the product per reduction; K = the rows below the block, flops
 * 2 * M * N * K with M the reflectors' count and N the columns of [V | C]),
 * taken while CTQR_PROFILE_UPDATE is enabled. */
ctqr_status ctqr_profile_read_reduction(int64_t *launches, double *total_ms, double *total_flops);

/* Phase timing (ctqr_profile_enable with the CTQR_PROFILE_PHASES bit): the
 * factorization and every direct solve record HIP events around their phases
 * on the stream they run on (never inside a graph capture, so the batched
 * solver's replays are not split).  ctqr_profile_phases returns, per phase,
 * the summed duration (ms; the caller must have synchronised the streams) and
 * the number of intervals; host synchronisation between phases counts in
 * none.  ms and count are host arrays of CTQR_NPHASES entries.
 * Factorization (Section II-C, "QR factorization"): */
#define CTQR_PHASE_PANEL         0   /* 32-column Householder panels (FP64 norms/reflectors) */
#define CTQR_PHASE_INNER         1   /* inner-panel T and updates inside a block column */
#define CTQR_PHASE_REDUCTION     2   /* [G | W] = V^T [V | C], block T, W' = T^T W */
#define CTQR_PHASE_UPDATE        3   /* trailing update C -= V W' of the rest of the matrix */
#define CTQR_PHASE_GROUP_UPDATE  4   /* update of the rest of a group by one of its blocks */
#define CTQR_PHASE_RINV          5   /* rank check and the stored diagonal-block inverses */
/* Solve (Eq. 4; Section II-C, "System solving") and its refinement: */
#define CTQR_PHASE_QTB           6   /* Q^T B */
#define CTQR_PHASE_TRSM          7   /* back substitution R X = (Q^T B)[0:n] */
#define CTQR_PHASE_RESIDUAL      8   /* FP64 sparse r = B - A X and s = A^T r */
#define CTQR_PHASE_REFINE_TRSM   9   /* R^T y = s and R d = y */
#define CTQR_PHASE_REFINE_OTHER 10   /* layout changes, X += d, convergence check */
#define CTQR_NPHASES            11
ctqr_status ctqr_profile_phases(double *ms, int64_t *count);

#ifdef __cplusplus
}
#endif
#endif /* CTQR_H */
