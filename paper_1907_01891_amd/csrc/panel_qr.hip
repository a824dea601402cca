// Panel factorization and compact-WY T build.
//
// Panel (the paper's Compute_dense_QR applied to one block column,
// Section II-C): unblocked Householder QR of a tall m_rem x w panel
// (w <= 32).  The panel's rows are split into contiguous slabs, one per
// workgroup, held in LDS in FP64 for the whole panel whatever the storage
// precision.  Reflector convention (LAPACK larfg):
// beta = -sign(alpha) ||[alpha; x]||, tau = (beta - alpha) / beta,
// v = [1; x / (alpha - beta)]; tau = 0 when x = 0.
//
// Two routes.  FP64 slabs first try the reconstruction route described
// further down (Cholesky QR twice, then the Householder vectors from an LU
// with sign choice: four grid barriers per panel); it gives the same V, tau
// and R up to rounding and hands the panel to the column route below when it
// is not safe.
//
// Column route, one grid barrier per column: after forming reflector j, each workgroup
// publishes its partial products w_c = v^T a_c for the columns c > j and,
// for column j+1, its partial sums S_aa = sum a^2, S_av = sum a v and
// S_vv = sum v^2 over the rows below the next pivot.  After the exchange
// every workgroup knows w and the squared norm of column j+1 after the
// update, S_aa - 2 tau w S_av + (tau w)^2 S_vv, so the next reflector needs
// no second exchange.  When that difference has cancelled below S_aa / 4
// (possible loss of digits) every workgroup instead takes the exact route:
// one more exchange of plain partial sums of squares of the updated column.
// The decision depends only on exchanged totals, so all workgroups take the
// same route.  Every cross-workgroup sum is taken in workgroup order, so the
// result is deterministic and identical in every workgroup.  The kernel
// also leaves each workgroup's partial Gram matrix V^T V for the T build.
//
// T build (the "S factors" of Section II-C): for H_1 ... H_w = I - V T V^T,
// T is upper triangular with T_jj = tau_j and
// T(0:j, j) = -tau_j T(0:j, 0:j) G(0:j, j), G = V^T V (the larft recurrence).
// Taken 32 columns at a time the recurrence reads
// T(0:32q, q) = -T(0:32q, 0:32q) (G(0:32q, q) T_qq), whose row block p only
// involves row block p of T, so one workgroup per row block builds it alone.
#include <cstdlib>
#include <cstring>
#include <algorithm>
#include <mutex>
#include "common.h"
#include "kernels.h"

namespace {

constexpr int PNT = 256;          // threads per panel workgroup
constexpr int PW = 32;            // max panel width
constexpr int PS = PANEL_XCH_STRIDE;   // per-workgroup exchange slots (see below)
// exchange slots: [0, 32) partial w_c for c = j+1+slot; 32: S_aa; 33: S_av;
// 34: S_vv; 35, 36: a(p+1, j+1) and v(p+1) before the update (workgroup 0)
constexpr int X_SAA = 32, X_SAV = 33, X_SVV = 34, X_A1 = 35, X_V1 = 36, X_N = 37;

__device__ inline double block_sum(double v, double *red)
{
    // Deterministic sum over the 256 threads: butterfly within each wave,
    // then the four wave sums in wave order.
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    if (threadIdx.x % CTQR_WAVE == 0) red[threadIdx.x / CTQR_WAVE] = v;
    __syncthreads();
    double r = red[0];
#pragma unroll
    for (int w = 1; w < PNT / CTQR_WAVE; ++w) r += red[w];
    __syncthreads();
    return r;
}

// Rows of a slab per lane (a wave covers a column, 64 rows at a time): the
// slab capacities below keep every slab within these many rows per lane.
template <typename SL> constexpr int rows_per_lane() { return sizeof(SL) == 8 ? 9 : 19; }

__device__ inline double wave_sum(double v)
{
    // deterministic butterfly over the 64 lanes (every lane gets the total)
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// ---------------------------------------------------------------------------
// Reconstruction route for FP64 slabs (four grid barriers per panel instead
// of one per column).  The panel P (rows r0 .. m-1, w columns) is first
// orthogonalised twice by Cholesky QR: G1 = P^T P = R1^T R1, Q1 = P R1^-1,
// G2 = Q1^T Q1 = R2^T R2, Q = Q1 R2^-1, R = R2 R1.  The Householder vectors
// follow from Q by the reconstruction of Ballard et al. (2015): the unit
// lower trapezoidal V and the upper triangular U' of the LU factorisation
// Q - [D; 0] = V U', with D = diag(d_j) chosen during the elimination as
// d_j = -sign(q_jj) of the current pivot element, so every pivot has modulus
// at least 1.  Then I - V T V^T with T = -U' D V_1^-T reproduces the
// factorisation: tau_j = -U'_jj d_j and the R of the Householder form is
// D R.  In exact arithmetic V, tau and D R are the vectors, scalars and R of
// the column-at-a-time route (beta = -sign(alpha) ||x||), so the two routes
// agree to rounding.  Rows below the top block: V = Q1 (U' R2)^-1.
//
// The route is taken only where it is safe, decided from exchanged totals so
// that every workgroup takes the same branch: every column has a nonzero
// part below its diagonal (the other route gives tau = 0 there), the first
// Cholesky factorisation has positive finite pivots, and after the first
// pass max |G2 - I| <= 1e-4 (a panel whose condition number is far below
// u^-1/2, where two passes leave Q orthonormal to rounding).  Otherwise the
// column-at-a-time route runs on the original panel.
// ---------------------------------------------------------------------------
constexpr int CQ_NE = 1056;          // exchanged partials per workgroup: Gram 32 x 32 (row-major) + 32 sums
constexpr int CQ_ML = 34;            // leading dimension of the 32 x 32 LDS matrices (16-byte aligned columns)
constexpr int CQ_MAT = 32 * CQ_ML;
constexpr int CQ_T1 = 0, CQ_T2 = CQ_NE, CQ_QT = 2 * CQ_NE;   // totals of the two passes, Q1's top rows
constexpr int CQ_TOT = CQ_QT + 32 * 32;
constexpr int CQ_NMAT = 7;           // R1, R2, LU, P, R and two inverses
constexpr int CQ_BUF = 192;          // row broadcasts (double-buffered) and pivots of the small factorisations
constexpr size_t CQ_LDS = (size_t)(CQ_NMAT * CQ_MAT + 64 + CQ_BUF) * sizeof(double);  // + signs, sums
constexpr size_t CQ_LDS_LIMIT = 156 * 1024;                  // slab + CQ_LDS, plus ~3 KiB static LDS
constexpr double CQ_ORTH_TOL = 1e-4;

__device__ __attribute__((always_inline)) inline doublex4 mfma_f64(double a, double b, doublex4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Gram matrix of the 32 columns val(rr, c) over the rows rr < nrows on FP64
// MFMA (v_mfma_f64_16x16x4f64: lane l supplies row k = l/16 of the 4-row
// step to column l%16 of each operand; output register r of lane l holds
// block entry (4r + l/16, l%16)).  Wave wv takes the 4-row steps at
// 16 t + 4 wv and feeds columns l%16 and 16 + l%16 to the blocks (0,0),
// (0,1) and (1,1); the four waves' sums are then added in wave order through
// scr (3072 doubles of LDS).  emit(i, j, g) receives every entry, the (1,0)
// block as the transpose of (0,1).
template <typename F, typename E>
__device__ __attribute__((always_inline)) inline void cq_gram(int nrows, F val, double *scr, E emit)
{
    const int wave = threadIdx.x / CTQR_WAVE, lane = threadIdx.x % CTQR_WAVE;
    const int li = lane % 16, kq = lane / 16;
    doublex4 g00 = {0.0, 0.0, 0.0, 0.0}, g01 = g00, g11 = g00;
    for (int k0 = 4 * wave; k0 < nrows; k0 += 16) {
        const int rr = k0 + kq;
        const bool in = rr < nrows;
        const int rc = in ? rr : nrows - 1;
        const double x0 = in ? val(rc, li) : 0.0, x1 = in ? val(rc, 16 + li) : 0.0;
        g00 = mfma_f64(x0, x0, g00);
        g01 = mfma_f64(x0, x1, g01);
        g11 = mfma_f64(x1, x1, g11);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        scr[(3 * wave + 0) * 256 + 64 * r + lane] = g00[r];
        scr[(3 * wave + 1) * 256 + 64 * r + lane] = g01[r];
        scr[(3 * wave + 2) * 256 + 64 * r + lane] = g11[r];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < 768; e += PNT) {
        const int b = e / 256, o = e % 256;
        double g = scr[b * 256 + o];
#pragma unroll
        for (int v = 1; v < PNT / CTQR_WAVE; ++v) g += scr[(3 * v + b) * 256 + o];
        const int i = 4 * ((o / 64) % 4) + (o % 64) / 16, j = o % 16;
        if (b == 0) {
            emit(i, j, g);
        } else if (b == 1) {
            emit(i, 16 + j, g);
            emit(16 + j, i, g);
        } else {
            emit(16 + i, 16 + j, g);
        }
    }
    __syncthreads();
}

// tot[e] = sum over the workgroups q < G of part[q * CQ_NE + e], e < ne (a
// multiple of 16).  One wave per 16 consecutive entries (a 128-byte line of
// every workgroup's partials); lane group l/16 sums the workgroups
// q = l/16 (mod 4) in increasing order, and the four group sums combine by a
// fixed butterfly, so the totals do not depend on timing.
__device__ __attribute__((always_inline)) inline void cq_reduce(const double *part, int G, int ne, double *tot)
{
    constexpr int NW = PNT / CTQR_WAVE, B = 16;
    const int wave = threadIdx.x / CTQR_WAVE, lane = threadIdx.x % CTQR_WAVE;
    const int e0 = lane % 16, grp = lane / 16;
    for (int line = blockIdx.x * NW + wave; line < ne / 16; line += gridDim.x * NW) {
        const int e = 16 * line + e0;
        double s = 0.0;
        for (int q0 = grp; q0 < G; q0 += 4 * B) {
            double v[B];
#pragma unroll
            for (int u = 0; u < B; ++u) {
                const int q = q0 + 4 * u;
                v[u] = q < G ? load_coherent(&part[(int64_t)q * CQ_NE + e]) : 0.0;
            }
#pragma unroll
            for (int u = 0; u < B; ++u) s += v[u];
        }
        s += __shfl_xor(s, 16);
        s += __shfl_xor(s, 32);
        if (lane < 16) store_coherent(&tot[e], s);
    }
}

// Orders one wave's LDS accesses across its lanes: a lane's read after the
// fence sees another lane's write before it (the compiler otherwise treats
// the lanes as independent threads and may hoist the read).
__device__ __attribute__((always_inline)) inline void wave_lds_fence()
{
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "workgroup");
    __builtin_amdgcn_wave_barrier();
}

// The three small factorisations below run in one wave with the 32 x 32
// matrix spread as half rows: lane l holds row i = l % 32, columns
// 16 h .. 16 h + 15 with h = l / 32, in 16 registers.  Their loops over the
// pivot index stay rolled: the panel kernel runs once per panel with a cold
// instruction cache, so compact code is faster than unrolled straight-line
// code here.  Rows are broadcast through buf (LDS) between wave fences.

// Cholesky factorisation G = R^T R of the leading w x w block of M
// (column-major, M[j * CQ_ML + i] = (i, j), both triangles present), in
// place (R in the upper triangle, zeros elsewhere in the 32 x 32 block), and
// X = R^-1 (same layout).  Right-looking on unscaled rows: step j publishes
// row j of the reduced matrix G' and row j of Z (Z = R^-T is built by the
// same elimination from I); rows i > j subtract (G'_ji / G'_jj) times both.
// Row j of R is G'_j / sqrt(G'_jj), row j of Z is Z_j / sqrt(G'_jj).  buf: 160
// doubles.  Returns false when a pivot is not positive and finite (the
// values left are then meaningless).
__device__ __attribute__((always_inline)) inline bool cq_cholesky_inv(double *M, int w, double *X, double *buf)
{
    const int lane = threadIdx.x % CTQR_WAVE, i = lane % 32, h = lane / 32;
    double g[16], z[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int k = 16 * h + t;
        g[t] = (i < w && k < w) ? M[k * CQ_ML + i] : 0.0;
        z[t] = (i == k && i < w) ? 1.0 : 0.0;
    }
    bool ok = true;
    double *diag = buf + 128;
    for (int j = 0; j < w; ++j) {
        // alternate halves: step j + 2 rewrites this half only after step
        // j + 1's fence, when every read of step j has completed
        double *b = buf + 64 * (j & 1);
        if (i == j)
#pragma unroll
            for (int t = 0; t < 16; ++t) {
                b[16 * h + t] = g[t];
                b[32 + 16 * h + t] = z[t];
            }
        wave_lds_fence();
        const double d = b[j];
        ok = ok && d > 0.0 && !isinf(d);
        const double invd = 1.0 / d;
        const double c = i > j ? b[i] * invd : 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t) {
            g[t] -= c * b[16 * h + t];
            z[t] -= c * b[32 + 16 * h + t];
        }
        if (lane == 0) diag[j] = sqrt(d);
    }
    wave_lds_fence();
    const double r = i < w ? diag[i] : 1.0, rs = 1.0 / r;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int k = 16 * h + t;
        const bool in = i < w && k < w;
        M[k * CQ_ML + i] = in ? (k > i ? g[t] * rs : (k == i ? r : 0.0)) : 0.0;
        X[i * CQ_ML + k] = in ? z[t] * rs : 0.0;      // X(k, i) = Z(i, k)
    }
    return ok;
}

// LU factorisation with the reconstruction's sign choice of the w x w block
// M (column-major), in place: the strict lower triangle becomes V's top block
// (unit diagonal implied), the upper triangle U'; dsign[j] = d_j.  Entries
// outside the w x w block stay 0.  Every step writes the current rows to a
// row-major scratch (32 x CQ_ML, S0 and S1 in turn), from which the pivot row
// and each row's entry in the pivot column are read; rows i > j then subtract
// l_i = S(i, j) / p_j times the pivot row.  buf: 32 doubles (the pivots).
__device__ __attribute__((always_inline)) inline void cq_lu_signs(double *M, int w, double *dsign, double *S0,
                                                                 double *S1, double *buf)
{
    const int lane = threadIdx.x % CTQR_WAVE, i = lane % 32, h = lane / 32;
    double a[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int k = 16 * h + t;
        a[t] = (i < w && k < w) ? M[k * CQ_ML + i] : 0.0;
    }
    for (int j = 0; j < w; ++j) {
        double *S = (j & 1) ? S1 : S0;         // alternate scratch, as in cq_cholesky_inv
#pragma unroll
        for (int t = 0; t < 16; ++t) S[i * CQ_ML + 16 * h + t] = a[t];
        wave_lds_fence();
        const double q = S[j * CQ_ML + j];
        const double d = q >= 0.0 ? -1.0 : 1.0;
        const double piv = q - d;                 // q + sign(q): modulus >= 1
        const double rp = 1.0 / piv;
        const double l = i > j ? S[i * CQ_ML + j] * rp : 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t) a[t] -= l * S[j * CQ_ML + 16 * h + t];
        if (lane == 0) {
            dsign[j] = d;
            buf[j] = piv;
        }
        if (h == 0 && i > j) M[j * CQ_ML + i] = l;       // column j of L
    }
    wave_lds_fence();
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int k = 16 * h + t;
        if (k >= i) M[k * CQ_ML + i] = (i < w && k < w) ? (k == i ? buf[i] : a[t]) : 0.0;
        else if (i >= w) M[k * CQ_ML + i] = 0.0;
    }
}

// X = U^-1 for the upper triangular leading w x w block of U (column-major),
// zeros elsewhere in the 32 x 32 block.  Gauss-Jordan from the last row up on
// unscaled rows (X starts as I): step j publishes row j, and rows i < j
// subtract (U_ij / U_jj) times it; row i is finally scaled by 1 / U_ii.
// LT: invert L^T instead, for the unit lower triangular L held strictly below
// the diagonal of U (L^T(i, j) = U[i * CQ_ML + j] for i < j, unit diagonal).
// buf: 64 doubles.
template <bool LT>
__device__ __attribute__((always_inline)) inline void cq_inverse(const double *U, int w, double *X, double *buf)
{
    const int lane = threadIdx.x % CTQR_WAVE, i = lane % 32, h = lane / 32;
    double x[16];
#pragma unroll
    for (int t = 0; t < 16; ++t) x[t] = (i == 16 * h + t && i < w) ? 1.0 : 0.0;
    for (int j = w - 1; j >= 0; --j) {
        double *b = buf + 32 * (j & 1);         // alternate halves, as in cq_cholesky_inv
        if (i == j)
#pragma unroll
            for (int t = 0; t < 16; ++t) b[16 * h + t] = x[t];
        wave_lds_fence();
        const double ujj = LT ? 1.0 : 1.0 / U[j * CQ_ML + j];
        const double c = i < j ? (LT ? U[i * CQ_ML + j] : U[j * CQ_ML + i]) * ujj : 0.0;
#pragma unroll
        for (int t = 0; t < 16; ++t) x[t] -= c * b[16 * h + t];
    }
    wave_lds_fence();
    const double rs = i < w ? (LT ? 1.0 : 1.0 / U[i * CQ_ML + i]) : 0.0;
#pragma unroll
    for (int t = 0; t < 16; ++t) {
        const int k = 16 * h + t;
        X[k * CQ_ML + i] = (i < w && k < w) ? x[t] * rs : 0.0;
    }
}

// T = -(U' D) L^-T, the compact-WY factor of the panel's reflectors
// (I - V T V^T = H_1 ... H_w): from Q D - [I; 0] = V U' D = -V T V_1^T with
// V_1 = L.  Stored in storage precision, column-major with leading dimension
// 32 (the w x w block, zeros below the diagonal).  Wave wv forms block
// (wv / 2, wv % 2) with eight v_mfma_f64_16x16x4f64.
template <typename TS>
__device__ __attribute__((always_inline)) inline void cq_store_t(const double *LU, const double *dsg, const double *Lt,
                                                                int w, TS *T)
{
    const int wave = threadIdx.x / CTQR_WAVE, lane = threadIdx.x % CTQR_WAVE;
    const int bi = 16 * (wave / 2), bj = 16 * (wave % 2);
    const int li = lane % 16, kq = lane / 16;
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < 32; k0 += 4) {
        const int k = k0 + kq;
        const double a = (k >= bi + li && k < w) ? LU[k * CQ_ML + bi + li] * dsg[k] : 0.0;
        acc = mfma_f64(a, Lt[(bj + li) * CQ_ML + k], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int i = bi + 4 * r + kq, j = bj + li;
        if (i < w && j < w) T[j * PW + i] = (TS)(0.0 - acc[r]);
    }
}

// C = triu(X) Y for 32 x 32 column-major LDS matrices (entries of X below
// its diagonal taken as 0).  Wave wv forms block (wv / 2, wv % 2) with eight
// v_mfma_f64_16x16x4f64.
__device__ __attribute__((always_inline)) inline void cq_upper_product(const double *X, const double *Y, double *C)
{
    const int wave = threadIdx.x / CTQR_WAVE, lane = threadIdx.x % CTQR_WAVE;
    const int bi = 16 * (wave / 2), bj = 16 * (wave % 2);
    const int li = lane % 16, kq = lane / 16;
    doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int k0 = 0; k0 < 32; k0 += 4) {
        const int k = k0 + kq;
        const double a = k >= bi + li ? X[k * CQ_ML + bi + li] : 0.0;
        acc = mfma_f64(a, Y[(bj + li) * CQ_ML + k], acc);
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) C[(bj + li) * CQ_ML + bi + 4 * r + kq] = acc[r];
}

// Rows [0, nrows) of the column-major matrix S (leading dimension lds, w
// columns): S := S X for X 32 x 32 in LDS (zero outside w x w), on FP64
// MFMA.  Wave wv takes the 16-row blocks wv, wv + 4, ...; each block's
// 16 x 32 inputs are read before any of its outputs is stored.
__device__ __attribute__((always_inline)) inline void cq_apply_right(double *S, int lds, int nrows, int w,
                                                                    const double *X)
{
    const int wave = threadIdx.x / CTQR_WAVE, lane = threadIdx.x % CTQR_WAVE;
    const int li = lane % 16, kq = lane / 16;
    double b0[8], b1[8];
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        b0[s] = X[li * CQ_ML + 4 * s + kq];
        b1[s] = X[(16 + li) * CQ_ML + 4 * s + kq];
    }
    for (int rb = 16 * wave; rb < nrows; rb += 16 * (PNT / CTQR_WAVE)) {
        const int r = rb + li;
        const int rc = r < nrows ? r : nrows - 1;
        double a[8];
#pragma unroll
        for (int s = 0; s < 8; ++s) a[s] = (r < nrows && 4 * s + kq < w) ? S[(4 * s + kq) * lds + rc] : 0.0;
        doublex4 c0 = {0.0, 0.0, 0.0, 0.0}, c1 = c0;
#pragma unroll
        for (int s = 0; s < 8; ++s) {
            c0 = mfma_f64(a[s], b0[s], c0);
            c1 = mfma_f64(a[s], b1[s], c1);
        }
#pragma unroll
        for (int q = 0; q < 4; ++q) {
            const int ro = rb + 4 * q + kq;
            if (ro < nrows) {
                if (li < w) S[li * lds + ro] = c0[q];
                if (16 + li < w) S[(16 + li) * lds + ro] = c1[q];
            }
        }
    }
}

__device__ __attribute__((always_inline)) inline bool wave_all(bool v)
{
    int x = v ? 1 : 0;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x &= __shfl_xor(x, o);
    return x != 0;
}

// Slab <- the panel's rows [row0, row0 + nrows) (column-major A:
// consecutive threads on consecutive rows).
template <typename TS, typename SL>
__device__ __attribute__((always_inline)) inline void load_slab(const TS *A, int64_t lda, int r0, int w, int row0,
                                                               int nrows, int ldsl, SL *slab)
{
    for (int idx = threadIdx.x; idx < nrows * w; idx += PNT) {
        const int c = idx / nrows, rr = idx % nrows;
        slab[c * ldsl + rr] = (SL)A[(int64_t)(r0 + c) * lda + row0 + rr];
    }
}

// The reconstruction route on an FP64 slab (described above).  On success the
// slab holds R (top rows of workgroup 0, on and above the diagonal) and the
// Householder vectors below it, and tau_s the scalars; returns false, with
// the slab holding the original panel, when the route is not safe.  Every
// workgroup returns the same value.  Workgroup 0 also stores the panel's
// compact-WY factor T to Tin.  ext: CQ_LDS bytes of LDS; cq_part: CQ_NE
// doubles per workgroup; cq_tot: CQ_TOT doubles.
template <typename TS>
__device__ __attribute__((always_inline)) bool cq_route(const TS *A, int64_t lda, int r0, int w, int row0,
                                                        int nrows, double *slab, int ldsl, double *ext, double *tau_s,
                                                        double *cq_part, double *cq_tot, TS *Tin, unsigned *bar,
                                                        unsigned &epoch, ctqr_info *info)
{
    const int G = gridDim.x, wg = blockIdx.x, tid = threadIdx.x;
    const int lane = tid % CTQR_WAVE, wave = tid / CTQR_WAVE;
    double *R1 = ext, *R2 = ext + CQ_MAT, *LU = ext + 2 * CQ_MAT, *P = ext + 3 * CQ_MAT, *R = ext + 4 * CQ_MAT;
    double *X = ext + 5 * CQ_MAT, *Lt = ext + 6 * CQ_MAT;
    double *dsg = ext + CQ_NMAT * CQ_MAT, *sub = dsg + 32, *buf = sub + 32;
    double *scr = LU;                  // Gram scratch: LU, P and R are free while the Grams run
    __shared__ int ok_s;
    double *mine = cq_part + (int64_t)wg * CQ_NE;
    auto slab_val = [&](int rr, int c) { return c < w ? slab[c * ldsl + rr] : 0.0; };
    auto emit_part = [&](int i, int j, double g) { store_coherent(&mine[32 * i + j], g); };

    // pass 1: partial Gram P^T P and, per column, the partial sum of squares
    // below the diagonal
    cq_gram(nrows, slab_val, scr, emit_part);
#pragma unroll
    for (int q = 0; q < 32 / (PNT / CTQR_WAVE); ++q) {
        const int c = wave + (PNT / CTQR_WAVE) * q;
        double s = 0.0;
        if (c < w)
            for (int rr = lane; rr < nrows; rr += CTQR_WAVE)
                if (row0 + rr > r0 + c) {
                    const double x = slab[c * ldsl + rr];
                    s += x * x;
                }
        s = wave_sum(s);
        if (lane == 0) store_coherent(&mine[1024 + c], s);
    }
    grid_barrier(bar, epoch, info);
    cq_reduce(cq_part, G, CQ_NE, cq_tot + CQ_T1);
    grid_barrier(bar, epoch, info);
    for (int e = tid; e < 1024; e += PNT) R1[(e % 32) * CQ_ML + e / 32] = load_coherent(&cq_tot[CQ_T1 + e]);
    if (tid < 32) sub[tid] = load_coherent(&cq_tot[CQ_T1 + 1024 + tid]);
    __syncthreads();
    if (wave == 0) {
        const double sc = sub[min(lane, 31)];
        bool ok = wave_all(lane >= w || (sc > 0.0 && !isinf(sc)));
        ok = cq_cholesky_inv(R1, w, X, buf) && ok;
        if (lane == 0) ok_s = ok;
    }
    __syncthreads();
    if (!ok_s) return false;

    // Q1 = P R1^-1; workgroup 0 publishes Q1's top rows; pass 2: Q1^T Q1
    cq_apply_right(slab, ldsl, nrows, w, X);
    __syncthreads();
    if (wg == 0)
        for (int e = tid; e < 1024; e += PNT) {
            const int rr = e / 32, c = e % 32;
            store_coherent(&cq_tot[CQ_QT + e], (rr < w && c < w) ? slab[c * ldsl + rr] : 0.0);
        }
    cq_gram(nrows, slab_val, scr, emit_part);
    grid_barrier(bar, epoch, info);
    cq_reduce(cq_part, G, 1024, cq_tot + CQ_T2);
    grid_barrier(bar, epoch, info);
    for (int e = tid; e < 1024; e += PNT) {
        R2[(e % 32) * CQ_ML + e / 32] = load_coherent(&cq_tot[CQ_T2 + e]);
        LU[(e % 32) * CQ_ML + e / 32] = load_coherent(&cq_tot[CQ_QT + e]);   // Q1 top row e/32, column e%32
    }
    __syncthreads();
    if (wave == 0) {
        bool ok = true;
        if (lane < w)
            for (int i = 0; i <= lane; ++i) {
                const double dev = fabs(R2[lane * CQ_ML + i] - (i == lane ? 1.0 : 0.0));
                ok = ok && dev <= CQ_ORTH_TOL;
            }
        ok = wave_all(ok);
        ok = cq_cholesky_inv(R2, w, X, buf) && ok;
        if (lane == 0) ok_s = ok;
    }
    __syncthreads();
    if (!ok_s) {
        load_slab(A, lda, r0, w, row0, nrows, ldsl, slab);
        __syncthreads();
        return false;
    }

    // Q's top block = Q1's top rows R2^-1, then its LU with the sign choice
    cq_apply_right(LU, CQ_ML, w, w, X);
    __syncthreads();
    if (wave == 0) cq_lu_signs(LU, w, dsg, P, R, buf);
    __syncthreads();
    if (wave == 0) cq_inverse<false>(LU, w, P, buf);                    // U'^-1
    else if (wave == 1 && wg == 0) cq_inverse<true>(LU, w, Lt, buf + 64);   // L^-T
    __syncthreads();
    cq_upper_product(R2, R1, R);              // R2 R1
    if (wg == 0) cq_store_t(LU, dsg, Lt, w, Tin);
    __syncthreads();
    cq_upper_product(X, P, R1);               // (U' R2)^-1 = R2^-1 U'^-1
    if (tid < w) tau_s[tid] = -LU[tid * CQ_ML + tid] * dsg[tid];
    __syncthreads();
    // V = Q1 (U' R2)^-1 (workgroup 0's top rows are then replaced): D R on and
    // above the diagonal, V's top block below it
    cq_apply_right(slab, ldsl, nrows, w, R1);
    __syncthreads();
    if (wg == 0)
        for (int e = tid; e < w * w; e += PNT) {
            const int rr = e % w, c = e / w;
            slab[c * ldsl + rr] = rr <= c ? dsg[rr] * R[c * CQ_ML + rr] : LU[c * CQ_ML + rr];
        }
    __syncthreads();
    return true;
}

// SL: element type of the slab.  FP64 whenever it fits in LDS; for very tall
// FP32 panels (more rows per workgroup than an FP64 slab can hold) an FP32
// slab, with every sum, norm and reflector scalar still formed in FP64.
// The slab is column-major (column c of the workgroup's rows at
// slab + c * rows_per_wg): the per-column products and updates give one wave
// to a column, its 64 lanes on consecutive rows, and each lane keeps the
// current reflector's values of its rows in registers.
__device__ inline void tb_diag(int q, int nb, const double (*Gq)[33], const double *__restrict__ tau,
                               double (*Tq)[33]);
constexpr size_t PANEL_T_LDS = 2 * 32 * 33 * sizeof(double);   // G and T of the column route's T build

template <typename TS, typename SL>
__global__ __launch_bounds__(PNT)
void panel_qr_kernel(TS *__restrict__ A, int64_t lda, int m, int r0, int w, int rows_per_wg,
                     double *__restrict__ tau_out, double *part, double *part2,
                     double *__restrict__ gram_part, int route, TS *__restrict__ Tin,
                     double *__restrict__ gram_sum, int want_t, unsigned *bar, ctqr_info *info)
{
    constexpr int NW = PNT / CTQR_WAVE;
    constexpr int RPL = rows_per_lane<SL>();
    extern __shared__ __attribute__((aligned(16))) unsigned char slab_raw[];
    SL *slab = reinterpret_cast<SL *>(slab_raw);  // column-major, column stride ldsl
    __shared__ double red[NW];
    __shared__ double wsum[PS];
    __shared__ double red4[NW][CTQR_WAVE];
    __shared__ double xch[PS];
    __shared__ double tau_s[PW];

    const int G = gridDim.x, wg = blockIdx.x, tid = threadIdx.x;
    const int lane = tid % CTQR_WAVE, wave = tid / CTQR_WAVE;
    const int ldsl = rows_per_wg;
    const int row0 = r0 + wg * rows_per_wg;
    const int nrows = max(0, min(rows_per_wg, m - row0));
    unsigned epoch = 0;

    load_slab(A, lda, r0, w, row0, nrows, ldsl, slab);
    __syncthreads();

    // pivot rows r0 .. r0+w-1 all lie in workgroup 0's slab (rows_per_wg >= 64)
    bool have = false;           // norm and alpha of column j known from the last exchange
    double ss = 0.0, alpha = 0.0;
    bool nonfinite = false;
    bool done = false;
    if constexpr (sizeof(SL) == sizeof(double)) {
        // the reconstruction route; its totals sit past this launch's
        // column-route exchange buffers
        if (route)
            done = cq_route<TS>(A, lda, r0, w, row0, nrows, reinterpret_cast<double *>(slab), ldsl,
                                reinterpret_cast<double *>(slab_raw + (size_t)ldsl * PW * sizeof(SL)), tau_s,
                                gram_part, part2 + (int64_t)2 * G * PS, Tin, bar, epoch, info);
    }
    for (int j = 0; j < (done ? 0 : w); ++j) {
        const int p = r0 + j;                     // pivot row
        SL *colj = slab + (int64_t)j * ldsl;
        if (!have) {
            double s = 0.0;
            for (int rr = tid; rr < nrows; rr += PNT)
                if (row0 + rr > p) {
                    double x = colj[rr];
                    s += x * x;
                }
            s = block_sum(s, red);
            if (tid == 0) {
                store_coherent(&part[wg], s);
                if (wg == 0) store_coherent(&part[G], colj[p - row0]);
            }
            grid_barrier(bar, epoch, info);
            double t = 0.0;
            for (int q = tid; q < G; q += PNT) t += load_coherent(&part[q]);
            ss = block_sum(t, red);
            alpha = load_coherent(&part[G]);
        }

        double tau = 0.0, beta = alpha, scale = 1.0;
        if (ss != 0.0) {
            double norm = sqrt(alpha * alpha + ss);
            beta = alpha >= 0.0 ? -norm : norm;
            tau = (beta - alpha) / beta;
            scale = 1.0 / (alpha - beta);
        }
        if (!(ss == ss) || !(alpha == alpha) || isinf(ss) || isinf(alpha)) nonfinite = true;
        if (tid == 0) tau_s[j] = tau;
        if (tau != 0.0)
            for (int rr = tid; rr < nrows; rr += PNT)
                if (row0 + rr > p) colj[rr] *= scale;
        __syncthreads();

        have = false;
        if (j + 1 < w) {
            double *x2 = part2 + (int64_t)(j & 1) * G * PS;    // alternate buffers by column
            // v on this lane's rows: 1 at the pivot, 0 above it and past the
            // slab.  Every slab read below is unconditional, with its row
            // clamped to the slab's last row (weight 0 there) and its column to
            // the panel's last, so the reads issue back to back instead of one
            // per branch.  nrows >= 1 in every launched workgroup.
            double vr[RPL];
#pragma unroll
            for (int k = 0; k < RPL; ++k) {
                const int rr = lane + CTQR_WAVE * k;
                const int g = row0 + rr;
                const double x = (double)colj[min(rr, nrows - 1)];
                vr[k] = (rr < nrows && g >= p) ? (g == p ? 1.0 : x) : 0.0;
            }
            // w_c = v^T a_c over this slab: wave wv takes columns j+1+wv+NW q,
            // q < PW / NW; all its products first, then all its wave sums
            constexpr int CPW = PW / NW;
            double acc[CPW];
#pragma unroll
            for (int q = 0; q < CPW; ++q) {
                const SL *col = slab + (int64_t)min(j + 1 + wave + NW * q, w - 1) * ldsl;
                acc[q] = 0.0;
#pragma unroll
                for (int k = 0; k < RPL; ++k) acc[q] += vr[k] * (double)col[min(lane + CTQR_WAVE * k, nrows - 1)];
            }
#pragma unroll
            for (int o = 32; o > 0; o >>= 1)
#pragma unroll
                for (int q = 0; q < CPW; ++q) acc[q] += __shfl_xor(acc[q], o);
            if (lane == 0)
#pragma unroll
                for (int q = 0; q < CPW; ++q) {
                    const int c = j + 1 + wave + NW * q;
                    if (c < w) wsum[c - (j + 1)] = acc[q];
                }
            // column j+1 below the next pivot: S_aa, S_av, S_vv (the last wave)
            if (wave == NW - 1) {
                const SL *col = slab + (int64_t)(j + 1) * ldsl;
                double saa = 0.0, sav = 0.0, svv = 0.0;
#pragma unroll
                for (int k = 0; k < RPL; ++k) {
                    const int rr = lane + CTQR_WAVE * k;
                    const double a0 = col[min(rr, nrows - 1)];
                    const bool in = rr < nrows && row0 + rr >= p + 2;
                    const double a = in ? a0 : 0.0, v = in ? vr[k] : 0.0;
                    saa += a * a;
                    sav += a * v;
                    svv += v * v;
                }
                saa = wave_sum(saa);
                sav = wave_sum(sav);
                svv = wave_sum(svv);
                if (lane == 0) {
                    wsum[X_SAA] = saa;
                    wsum[X_SAV] = sav;
                    wsum[X_SVV] = svv;
                }
            }
            __syncthreads();
            if (tid < X_A1 && (tid >= PW || j + 1 + tid < w)) store_coherent(&x2[(int64_t)wg * PS + tid], wsum[tid]);
            if (wg == 0 && tid == 0) {
                const int rr = p + 1 - row0;
                store_coherent(&x2[X_A1], slab[(int64_t)(j + 1) * ldsl + rr]);
                store_coherent(&x2[X_V1], colj[rr]);
            }
            grid_barrier(bar, epoch, info);

            // totals over the workgroups, in workgroup order
            {
                const int e = tid % CTQR_WAVE, grp = tid / CTQR_WAVE;
                constexpr int BATCH = 64;   // every load of up to 256 workgroups in flight
                double s = 0.0;
                if (e < X_A1 && (e >= PW || j + 1 + e < w))
                    for (int q0 = grp; q0 < G; q0 += NW * BATCH) {
                        // BATCH loads in flight, then summed in workgroup order
                        double v[BATCH];
#pragma unroll
                        for (int u = 0; u < BATCH; ++u) {
                            const int q = q0 + NW * u;
                            v[u] = q < G ? load_coherent(&x2[(int64_t)q * PS + e]) : 0.0;
                        }
#pragma unroll
                        for (int u = 0; u < BATCH; ++u) s += v[u];
                    }
                red4[grp][e] = s;
                __syncthreads();
                if (tid < X_A1) {
                    double t = red4[0][tid];
                    for (int q = 1; q < NW; ++q) t += red4[q][tid];
                    xch[tid] = t;
                }
                if (tid == X_A1 || tid == X_V1) xch[tid] = load_coherent(&x2[tid]);
                __syncthreads();
            }
            if (tau != 0.0) {
                // a_c -= (tau w_c) v, the columns of each wave as above
#pragma unroll
                for (int q = 0; q < CPW; ++q) {
                    const int c = j + 1 + wave + NW * q;
                    if (c < w) {
                        SL *col = slab + (int64_t)c * ldsl;
                        const double f = tau * xch[c - (j + 1)];
                        // every read first, then the stores of the lane's own rows
                        // (v = 0 above the pivot leaves those rows unchanged)
                        double nv[RPL];
#pragma unroll
                        for (int k = 0; k < RPL; ++k)
                            nv[k] = (double)col[min(lane + CTQR_WAVE * k, nrows - 1)] - f * vr[k];
#pragma unroll
                        for (int k = 0; k < RPL; ++k) {
                            const int rr = lane + CTQR_WAVE * k;
                            if (rr < nrows) col[rr] = (SL)nv[k];
                        }
                    }
                }
            }
            // squared norm below the next pivot and the next alpha, after the update
            const double tw = tau * xch[0];
            const double ssn = xch[X_SAA] - 2.0 * tw * xch[X_SAV] + tw * tw * xch[X_SVV];
            if (ssn >= 0.25 * xch[X_SAA]) {
                have = true;
                ss = ssn;
                alpha = xch[X_A1] - tw * xch[X_V1];
            }
        }
        if (wg == 0 && tid == 0) colj[p - row0] = (SL)beta;
        __syncthreads();
    }

    // write the factored slab back in storage precision
    for (int idx = tid; idx < nrows * w; idx += PNT) {
        int c = idx / nrows, rr = idx % nrows;
        A[(int64_t)(r0 + c) * lda + row0 + rr] = (TS)slab[c * ldsl + rr];
    }
    if (wg == 0 && tid < w) tau_out[tid] = tau_s[tid];
    if (nonfinite && tid == 0 && wg == 0) info_event(info, CTQR_NONFINITE, r0);

    // partial Gram V^T V over this slab (V unit lower trapezoidal), rounded to
    // storage precision first so it describes the stored vectors: a 32 x 32
    // product over the slab's rows on FP64 MFMA (v_mfma_f64_16x16x4f64), one
    // 16 x 16 block per wave.  Lane l feeds row k0 + l/16 of columns
    // bi + l%16 and bj + l%16; output register r of lane l holds
    // G(bi + 4r + l/16, bj + l%16).
    // After the reconstruction route T is already stored.
    if (done || !want_t) return;
    __syncthreads();
    auto vval = [&](int rr, int c) -> double {
        if (rr >= nrows || c >= w) return 0.0;
        const int g = row0 + rr;
        return g == r0 + c ? 1.0 : (g > r0 + c ? (double)(TS)slab[c * ldsl + rr] : 0.0);
    };
    {
        const int bi = 16 * (wave / 2), bj = 16 * (wave % 2);
        const int li = lane % 16, kq = lane / 16;
        doublex4 g4 = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < nrows; k0 += 4) {
            const double a = vval(k0 + kq, bi + li), b = vval(k0 + kq, bj + li);
            g4 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, g4, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
            store_coherent(&gram_part[(int64_t)wg * PW * PW + (bi + 4 * r + kq) + PW * (bj + li)], g4[r]);
    }
    // The Gram summed over the workgroups, 16 entries at a time per
    // workgroup: 16 threads per entry each sum every 16th partial, then the
    // 16 sums in thread order.
    grid_barrier(bar, epoch, info);
    double *gsum = &red4[0][0];   // 16 x 16
    {
        const int el = tid % 16, grp = tid / 16;
        for (int b = wg; b < PW * PW / 16; b += G) {
            double t = 0.0;
            for (int q = grp; q < G; q += 16) t += load_coherent(&gram_part[(int64_t)q * PW * PW + 16 * b + el]);
            gsum[16 * grp + el] = t;
            __syncthreads();
            if (tid < 16) {
                double u = 0.0;
                for (int q = 0; q < 16; ++q) u += gsum[16 * q + tid];
                store_coherent(&gram_sum[16 * b + tid], u);
            }
            __syncthreads();
        }
    }
    grid_barrier(bar, epoch, info);
    if (wg != 0) return;
    // T = (diag(1/tau) + striu(G))^-1 by the recurrence, in workgroup 0 (the
    // slab's LDS, at least PANEL_T_LDS bytes, is free now)
    double (*Gs)[33] = reinterpret_cast<double (*)[33]>(slab_raw);
    double (*Tq)[33] = Gs + 32;
    for (int e = tid; e < 1024; e += PNT) {
        const int i = e % 32, j = e / 32;
        Gs[i][j] = (i < w && j < w) ? load_coherent(&gram_sum[j * PW + i]) : 0.0;
    }
    __syncthreads();
    tb_diag(0, w, Gs, tau_s, Tq);
    __syncthreads();
    for (int e = tid; e < 1024; e += PNT) {
        const int i = e % 32, j = e / 32;
        if (i < w && j < w) Tin[j * PW + i] = (TS)Tq[i][j];
    }
}

// T from G and tau, one workgroup per 32-row block p of T.  Row block p
// depends only on G, tau and itself:
//   T_pp = the recurrence on (G_pp, tau_p),
//   T_pq = -sum_{k=p}^{q-1} T_pk (G_kq T_qq)   for q > p,
// so the workgroups run independently; each recomputes the diagonal blocks
// T_qq it needs.  All operands live in LDS; arithmetic is FP64.
constexpr int TB_MAXQ = 8;                  // nb <= 256
constexpr int TB_LD = 32 * TB_MAXQ + 1;

__device__ inline void tb_diag(int q, int nb, const double (*Gq)[33], const double *__restrict__ tau,
                               double (*Tq)[33])
{
    // one thread per row r of T_qq: T(r, r) = tau_r, T(r, j) = -tau_j sum_{c<j} T(r, c) G(c, j)
    const int r = threadIdx.x;
    if (r >= 32) return;
    const int gi = 32 * q + r;
    double t[32];
#pragma unroll
    for (int j = 0; j < 32; ++j) {
        const int gj = 32 * q + j;
        double val;
        if (gj >= nb || gi >= nb || j < r) {
            val = 0.0;
        } else if (j == r) {
            val = tau[gj];
        } else {
            double s = 0.0;
#pragma unroll
            for (int c = 0; c < j; ++c) s += t[c] * Gq[c][j];
            val = -tau[gj] * s;
        }
        t[j] = val;
    }
#pragma unroll
    for (int j = 0; j < 32; ++j) Tq[r][j] = t[j];
}

template <typename TG>
__device__ inline void tb_stage(int nb, const TG *__restrict__ Gm, int64_t ldg, int kb, int qb, double (*dst)[33])
{
    for (int e = threadIdx.x; e < 1024; e += 256) {
        int i = e % 32, j = e / 32;
        int gi = 32 * kb + i, gj = 32 * qb + j;
        dst[i][j] = (gi < nb && gj < nb) ? (double)Gm[(int64_t)gj * ldg + gi] : 0.0;
    }
}

template <typename TG, typename TT>
__global__ __launch_bounds__(256)
void tbuild_kernel(int nb, const TG *__restrict__ Gm, int64_t ldg, const double *__restrict__ tau,
                   TT *__restrict__ Tout, int64_t ldt, const double *__restrict__ skip)
{
    if (skip && *skip != 0.0) return;
    __shared__ double Trow[32][TB_LD];      // rows 32p .. 32p+31 of T, all nb columns
    __shared__ double Gs[32][33];
    __shared__ double Tq[32][33];
    __shared__ double Y[32][33];
    const int p = blockIdx.x, tid = threadIdx.x;
    const int nq = (nb + 31) / 32;

    for (int e = tid; e < 32 * TB_LD; e += 256) (&Trow[0][0])[e] = 0.0;
    tb_stage(nb, Gm, ldg, p, p, Gs);
    __syncthreads();
    tb_diag(p, nb, Gs, tau, Tq);
    __syncthreads();
    for (int e = tid; e < 1024; e += 256) Trow[e % 32][32 * p + e / 32] = Tq[e % 32][e / 32];
    __syncthreads();

    for (int q = p + 1; q < nq; ++q) {
        tb_stage(nb, Gm, ldg, q, q, Gs);
        __syncthreads();
        tb_diag(q, nb, Gs, tau, Tq);
        __syncthreads();
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = p; k < q; ++k) {
            tb_stage(nb, Gm, ldg, k, q, Gs);          // G_kq
            __syncthreads();
            for (int o = 0; o < 4; ++o) {             // Y = G_kq T_qq (T_qq upper triangular)
                int e = tid + 256 * o, i = e % 32, c = e / 32;
                double s = 0.0;
                for (int l = 0; l <= c; ++l) s += Gs[i][l] * Tq[l][c];
                Y[i][c] = s;
            }
            __syncthreads();
            for (int o = 0; o < 4; ++o) {             // acc += T_pk Y
                int e = tid + 256 * o, i = e % 32, c = e / 32;
                double s = 0.0;
                for (int l = 0; l < 32; ++l) s += Trow[i][32 * k + l] * Y[l][c];
                acc[o] += s;
            }
            __syncthreads();
        }
        for (int o = 0; o < 4; ++o) {
            int e = tid + 256 * o, i = e % 32, c = e / 32;
            Trow[i][32 * q + c] = -acc[o];
        }
        __syncthreads();
    }
    for (int e = tid; e < 32 * nb; e += 256) {
        int i = e % 32, j = e / 32;
        int gi = 32 * p + i;
        if (gi < nb) Tout[(int64_t)j * ldt + gi] = (TT)Trow[i][j];
    }
}

// Blocks wider than 32: first every diagonal block T_qq by the recurrence
// above (one workgroup each, FP64, to the workspace Tw), then every block
// column on its own.  With U = diag(1 / tau) + striu(G), T = U^-1 (the
// recurrence is the column-by-column form of that inverse), so
// U_pp T_pq = -sum_{k=p+1}^{q} G_pk T_kq, i.e.
// T_pq = -T_pp sum_{k=p+1}^{q} G_pk T_kq, for p = q-1 down to 0: each
// block column is a chain of q products of its own (FP64 MFMA, a 16 x 16
// output block per wave), and the block columns run in parallel.
template <typename TG>
__global__ __launch_bounds__(256)
void tbuild_diag_kernel(int nb, const TG *__restrict__ Gm, int64_t ldg, const double *__restrict__ tau,
                        double *__restrict__ Tw)
{
    __shared__ double Gs[32][33];
    __shared__ double Tq[32][33];
    const int q = blockIdx.x;
    tb_stage(nb, Gm, ldg, q, q, Gs);
    __syncthreads();
    tb_diag(q, nb, Gs, tau, Tq);
    __syncthreads();
    for (int e = threadIdx.x; e < 1024; e += 256) {
        const int i = e % 32, j = e / 32, gi = 32 * q + i, gj = 32 * q + j;
        if (gi < nb && gj < nb) Tw[(int64_t)gj * nb + gi] = Tq[i][j];
    }
}

constexpr size_t TB_COL_LDS = (size_t)(32 * TB_MAXQ * 33 + 32 * TB_LD + 2 * 32 * 33) * sizeof(double);

template <typename TG, typename TT>
__global__ __launch_bounds__(256)
void tbuild_col_kernel(int nb, const TG *__restrict__ Gm, int64_t ldg, const double *__restrict__ Tw,
                       TT *__restrict__ Tout, int64_t ldt)
{
    extern __shared__ __attribute__((aligned(16))) double tbsm[];
    double (*Tc)[33] = reinterpret_cast<double (*)[33]>(tbsm);                        // block column q, by rows
    double (*Gp)[TB_LD] = reinterpret_cast<double (*)[TB_LD]>(tbsm + 32 * TB_MAXQ * 33);   // row panel p of G
    double (*Tp)[33] = reinterpret_cast<double (*)[33]>(tbsm + 32 * TB_MAXQ * 33 + 32 * TB_LD);   // T_pp
    double (*Sx)[33] = Tp + 32;                                                       // the sum
    const int q = blockIdx.x, tid = threadIdx.x;
    // MFMA lanes: lane l feeds row l % 16 / column l % 16 and k = l / 16 of a
    // 4-deep step; its output register r is block entry (4 r + l / 16, l % 16)
    const int wv = tid / 64, l = tid % 64, li = l % 16, lk = l / 16;
    const int bi = wv % 2, bj = wv / 2;
    for (int e = tid; e < 1024; e += 256) {
        const int a = e % 32, b = e / 32, ga = 32 * q + a, gb = 32 * q + b;
        Tc[32 * q + a][b] = (ga < nb && gb < nb) ? Tw[(int64_t)gb * nb + ga] : 0.0;
    }
    // step p's operands (row panel p of G, T_pp) are loaded into registers
    // during step p + 1 and stored to LDS at the start of step p
    constexpr int GREG = 32 * 32 * (TB_MAXQ - 1) / 256;
    TG gr[GREG];
    double tr[4];
    auto fetch = [&](int p) {
        const int c0 = 32 * (p + 1), cw = 32 * (q - p);
#pragma unroll
        for (int u = 0; u < GREG; ++u) {
            const int e = tid + 256 * u, a = e % 32, gc = c0 + e / 32;
            if (e < 32 * cw) gr[u] = gc < nb ? Gm[(int64_t)gc * ldg + 32 * p + a] : TG(0);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u, a = e % 32, b = e / 32;
            tr[u] = Tw[(int64_t)(32 * p + b) * nb + 32 * p + a];
        }
    };
    if (q > 0) fetch(q - 1);
    for (int p = q - 1; p >= 0; --p) {
        const int c0 = 32 * (p + 1), cw = 32 * (q - p);
#pragma unroll
        for (int u = 0; u < GREG; ++u) {
            const int e = tid + 256 * u;
            if (e < 32 * cw) Gp[e % 32][e / 32] = (double)gr[u];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int e = tid + 256 * u;
            Tp[e % 32][e / 32] = tr[u];
        }
        __syncthreads();
        if (p > 0) fetch(p - 1);
        {
            // Sx = G_p,(p+1..q) T_(p+1..q),q on FP64 MFMA: wave wv the 16 x 16 block (bi, bj)
            doublex4 acc = {0.0, 0.0, 0.0, 0.0};
            for (int kk = 0; kk < cw; kk += 4)
                acc = mfma_f64(Gp[16 * bi + li][kk + lk], Tc[c0 + kk + lk][16 * bj + li], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) Sx[16 * bi + 4 * r + lk][16 * bj + li] = acc[r];
        }
        __syncthreads();
        {
            // T_pq = -T_pp Sx
            doublex4 acc = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int kk = 0; kk < 32; kk += 4)
                acc = mfma_f64(Tp[16 * bi + li][kk + lk], Sx[kk + lk][16 * bj + li], acc);
#pragma unroll
            for (int r = 0; r < 4; ++r) Tc[32 * p + 16 * bi + 4 * r + lk][16 * bj + li] = -acc[r];
        }
        __syncthreads();
    }
    for (int e = tid; e < 32 * nb; e += 256) {
        const int r = e % nb, b = e / nb, gb = 32 * q + b;
        if (gb < nb) Tout[(int64_t)gb * ldt + r] = r < 32 * q + 32 ? (TT)Tc[r][b] : TT(0);
    }
}

}  // namespace

int panel_rows_per_wg(int mrem, int ncu)
{
    int rows = (int)ceil_div(mrem, ncu);
    if (rows < 64) rows = 64;
    return rows;
}

// LDS of a slab of rows_per_wg rows (element size esz).  FP64 slabs keep to
// 144 KiB; the FP32 slab of very tall panels may take 152 KiB (the kernel's
// static LDS adds about 5 KiB; gfx950 offers 160 KiB per workgroup).
size_t panel_lds_bytes(int rows_per_wg, size_t esz) { return (size_t)rows_per_wg * PW * esz; }

// at most 64 rows_per_lane rows per slab, the register tile of the per-column steps
int panel_max_rows_per_wg() { return std::min((int)((144 * 1024) / (PW * sizeof(double))), 64 * rows_per_lane<double>()); }
int panel_max_rows_per_wg_f32() { return std::min((int)((152 * 1024) / (PW * sizeof(float))), 64 * rows_per_lane<float>()); }

template <typename TS>
ctqr_status panel_qr(TS *A, int64_t lda, int m, int r0, int w, double *tau, double *part,
                     double *part2, double *gram_part, double *gram, TS *Tin, bool want_t, unsigned *bar,
                     ctqr_info *info, int ncu, hipStream_t st)
{
    const int mrem = m - r0;
    const int rows = panel_rows_per_wg(mrem, ncu);
    const bool f32slab = sizeof(TS) == 4 && rows > panel_max_rows_per_wg();
    if (rows > (f32slab ? panel_max_rows_per_wg_f32() : panel_max_rows_per_wg())) return CTQR_EUNSUPPORTED;
    const int G = (int)ceil_div(mrem, rows);
    size_t lds = panel_lds_bytes(rows, f32slab ? sizeof(float) : sizeof(double));
    // the reconstruction route: FP64 slabs with room for its LDS, at most 256
    // workgroups (its exchange sits past the column route's), more panel rows
    // than columns; CTQR_PANEL_ROUTE=columns keeps the column-at-a-time route
    const char *ev = getenv("CTQR_PANEL_ROUTE");
    int route = !f32slab && !(ev && !strcmp(ev, "columns")) && G <= 256 && mrem > w &&
                lds + CQ_LDS <= CQ_LDS_LIMIT;
    if (route) lds += CQ_LDS;
    lds = std::max(lds, PANEL_T_LDS);
    int wt = want_t ? 1 : 0;
    void *args[] = {&A,         (void *)&lda, &m,   &r0,   &w,  (void *)&rows, &tau, &part, &part2,
                    &gram_part, &route,       &Tin, &gram, &wt, &bar,          &info};
    if (f32slab)
        HIP_TRY(hipLaunchCooperativeKernel((const void *)panel_qr_kernel<TS, float>, dim3(G), dim3(PNT), args, lds,
                                           st));
    else
        HIP_TRY(hipLaunchCooperativeKernel((const void *)panel_qr_kernel<TS, double>, dim3(G), dim3(PNT), args,
                                           lds, st));
    return CTQR_OK;
}

ctqr_status panel_setup(int max_rows)
{
    const int l64 = (int)std::max(panel_lds_bytes(max_rows, sizeof(double)), CQ_LDS_LIMIT);
    const int l32 = (int)panel_lds_bytes(panel_max_rows_per_wg_f32(), sizeof(float));
    HIP_TRY(hipFuncSetAttribute((const void *)panel_qr_kernel<float, double>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, l64));
    HIP_TRY(hipFuncSetAttribute((const void *)panel_qr_kernel<double, double>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, l64));
    HIP_TRY(hipFuncSetAttribute((const void *)panel_qr_kernel<float, float>,
                                hipFuncAttributeMaxDynamicSharedMemorySize, l32));
    return CTQR_OK;
}

template <typename TG, typename TT>
ctqr_status tbuild(int nb, const TG *G, int64_t ldg, const double *tau, TT *T, int64_t ldt, double *Tw,
                   hipStream_t st, const double *skip)
{
    if (nb < 1 || nb > 32 * TB_MAXQ) return CTQR_EINVAL;
    if (nb <= 32 || Tw == nullptr) {
        LAUNCH_TRY((tbuild_kernel<TG, TT>), dim3((unsigned)ceil_div(nb, 32)), dim3(256), 0, st, nb, G, ldg, tau, T,
                   ldt, skip);
        return CTQR_OK;
    }
    if (skip) return CTQR_EINVAL;          // (only the 32-wide inner T build is skippable)
    static std::once_flag once;
    static hipError_t attr = hipSuccess;
    std::call_once(once, [] {
        attr = hipFuncSetAttribute((const void *)tbuild_col_kernel<TG, TT>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)TB_COL_LDS);
    });
    HIP_TRY(attr);
    const unsigned nq = (unsigned)ceil_div(nb, 32);
    LAUNCH_TRY((tbuild_diag_kernel<TG>), dim3(nq), dim3(256), 0, st, nb, G, ldg, tau, Tw);
    LAUNCH_TRY((tbuild_col_kernel<TG, TT>), dim3(nq), dim3(256), TB_COL_LDS, st, nb, G, ldg, (const double *)Tw, T,
               ldt);
    return CTQR_OK;
}

template ctqr_status panel_qr<float>(float *, int64_t, int, int, int, double *, double *, double *,
                                     double *, double *, float *, bool, unsigned *, ctqr_info *, int, hipStream_t);
template ctqr_status panel_qr<double>(double *, int64_t, int, int, int, double *, double *, double *,
                                      double *, double *, double *, bool, unsigned *, ctqr_info *, int,
                                      hipStream_t);
template ctqr_status tbuild<double, float>(int, const double *, int64_t, const double *, float *, int64_t,
                                           double *, hipStream_t,
                                           const double *);
template ctqr_status tbuild<double, double>(int, const double *, int64_t, const double *, double *, int64_t,
                                            double *, hipStream_t,
                                           const double *);
template ctqr_status tbuild<float, float>(int, const float *, int64_t, const double *, float *, int64_t,
                                          double *, hipStream_t,
                                           const double *);
