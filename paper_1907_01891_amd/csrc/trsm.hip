// Block triangular solves with the R factor (Section II-C, "System solving":
// the block-row backward substitution of Trsm_lunn / Gemm_nn_mo tasks).
//
//   trsm_upper:        R X = C, block rows from the bottom:
//                      X_i = R_ii^-1 C_i;  C_{0:i} -= R_{0:i, i} X_i
//   trsm_upper_trans:  R^T Y = C, block rows from the top (used by the
//                      refinement's semi-normal equations):
//                      Y_i = R_ii^-T C_i;  C_{i+1:} -= R_{i, i+1:}^T Y_i
//
// The diagonal blocks R_ii are TRSM_BIG (2048) wide, so a solve is a chain of
// n / 2048 steps, each two large MFMA products.  Their inverses are built
// once per solve: 256 x 256 diagonal inverses by trinv_kernel, then doubled to
// 512, 1024 and 2048 with inv([A B; 0 D]) = [inv(A), -inv(A) B inv(D); 0,
// inv(D)] as MFMA products.
//
// trinv_kernel: row block p (32 rows) of inv(U), U upper triangular, depends
// only on U and on itself: X_pp = inv(U_pp), X_pq = -(sum_{k=p}^{q-1} X_pk
// U_kq) X_qq, so each 32-row block is built by its own workgroup (FP64,
// operands in LDS), each recomputing the small diagonal inverses X_qq it
// needs.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int BT = TRSM_BASE;          // block inverted by trinv_kernel
constexpr int BIG = TRSM_BIG;          // diagonal block of the substitutions
constexpr int RB = 32;                 // row block of the inversion
constexpr int NQ = BT / RB;            // row blocks per base block
constexpr int XLD = BT + 1;

// Rs <- R(base + 32*kb .., base + 32*qb ..) as a 32 x 32 FP64 tile (zero
// outside the n x n matrix)
template <typename T>
__device__ inline void stage_r(int n, const T *__restrict__ R, int64_t ldr, int base, int kb, int qb,
                               double (*Rs)[33])
{
    for (int e = threadIdx.x; e < 1024; e += 256) {
        int i = e % 32, j = e / 32;
        int gi = base + 32 * kb + i, gj = base + 32 * qb + j;
        Rs[i][j] = (gi < n && gj < n) ? (double)R[(int64_t)gj * ldr + gi] : 0.0;
    }
}

// Xq <- inv(Rs) for an upper-triangular 32 x 32 tile: thread c builds column
// c by back substitution (columns past the matrix edge are zero).
__device__ inline void inv32(const double (*Rs)[33], double (*Xq)[33], int valid)
{
    const int c = threadIdx.x;
    if (c >= 32) return;
    double x[32];
#pragma unroll
    for (int i = 31; i >= 0; --i) {
        double v = 0.0;
        if (i <= c && c < valid) {
            double s = (i == c) ? 1.0 : 0.0;
#pragma unroll
            for (int k = i + 1; k < 32; ++k)
                if (k <= c) s -= Rs[i][k] * x[k];
            v = s / Rs[i][i];
        }
        x[i] = v;
    }
#pragma unroll
    for (int i = 0; i < 32; ++i) Xq[i][c] = x[i];
}

// inv of the 256 x 256 diagonal block blk of R, row block p, written into
// the BIG-wide inverse array (column j of the matrix at Rinv + j * BIG, row
// (j's block offset inside its BIG block) + i).
template <typename T>
__global__ __launch_bounds__(256)
void trinv_kernel(int n, const T *__restrict__ R, int64_t ldr, T *__restrict__ Rinv, int blk0)
{
    __shared__ double Xrow[RB][XLD];
    __shared__ double Rs[32][33];
    __shared__ double Xq[32][33];
    __shared__ double Y[32][33];
    const int blk = blk0 + (int)blockIdx.x, p = blockIdx.y, tid = threadIdx.x;
    const int base = blk * BT;
    const int nbk = min(BT, n - base);
    const int nq = (nbk + RB - 1) / RB;
    if (p >= nq) return;
    for (int e = tid; e < RB * XLD; e += 256) (&Xrow[0][0])[e] = 0.0;
    stage_r(n, R, ldr, base, p, p, Rs);
    __syncthreads();
    inv32(Rs, Xq, nbk - RB * p);
    __syncthreads();
    for (int e = tid; e < 1024; e += 256) Xrow[e % 32][RB * p + e / 32] = Xq[e % 32][e / 32];
    __syncthreads();
    for (int q = p + 1; q < nq; ++q) {
        double acc[4] = {0.0, 0.0, 0.0, 0.0};
        for (int k = p; k < q; ++k) {
            stage_r(n, R, ldr, base, k, q, Rs);        // U_kq
            __syncthreads();
            for (int o = 0; o < 4; ++o) {
                int e = tid + 256 * o, i = e % 32, c = e / 32;
                double s = 0.0;
                for (int l = 0; l < 32; ++l) s += Xrow[i][RB * k + l] * Rs[l][c];
                acc[o] += s;
            }
            __syncthreads();
        }
        for (int o = 0; o < 4; ++o) {
            int e = tid + 256 * o;
            Y[e % 32][e / 32] = acc[o];
        }
        stage_r(n, R, ldr, base, q, q, Rs);
        __syncthreads();
        inv32(Rs, Xq, nbk - RB * q);
        __syncthreads();
        for (int o = 0; o < 4; ++o) {                  // X_pq = -Y X_qq
            int e = tid + 256 * o, i = e % 32, c = e / 32;
            double s = 0.0;
            for (int l = 0; l <= c; ++l) s += Y[i][l] * Xq[l][c];
            Xrow[i][RB * q + c] = -s;
        }
        __syncthreads();
    }
    const int off = base % BIG;
    for (int e = tid; e < RB * nbk; e += 256) {
        int i = e % RB, j = e / RB;
        Rinv[(int64_t)(base + j) * BIG + off + RB * p + i] = (T)Xrow[i][j];
    }
}

// max/min |R_kk| and the first k with |R_kk| <= n * u * max|R_ii| (u of the
// storage precision), or a non-finite diagonal.  One workgroup.
template <typename T>
__global__ __launch_bounds__(1024)
void rdiag_kernel(int n, const T *__restrict__ R, int64_t ldr, ctqr_info *info)
{
    __shared__ double smax[1024], smin[1024];
    __shared__ int sbad[1024];
    double mx = 0.0, mn = INFINITY;
    bool nonfin = false;
    for (int k = threadIdx.x; k < n; k += 1024) {
        double d = fabs((double)R[(int64_t)k * ldr + k]);
        if (!(d <= 1e300)) nonfin = true;
        mx = fmax(mx, d);
        mn = fmin(mn, d);
    }
    smax[threadIdx.x] = mx;
    smin[threadIdx.x] = mn;
    sbad[threadIdx.x] = nonfin ? 1 : 0;
    __syncthreads();
    for (int s = 512; s > 0; s >>= 1) {
        if (threadIdx.x < s) {
            smax[threadIdx.x] = fmax(smax[threadIdx.x], smax[threadIdx.x + s]);
            smin[threadIdx.x] = fmin(smin[threadIdx.x], smin[threadIdx.x + s]);
            sbad[threadIdx.x] |= sbad[threadIdx.x + s];
        }
        __syncthreads();
    }
    const double u = sizeof(T) == 4 ? 5.96e-8 : 1.11e-16;
    const double thr = (double)n * u * smax[0];
    __shared__ int first;
    if (threadIdx.x == 0) first = n;
    __syncthreads();
    for (int k = threadIdx.x; k < n; k += 1024) {
        double d = fabs((double)R[(int64_t)k * ldr + k]);
        if (d <= thr) atomicMin(&first, k);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        info->rdiag_max = smax[0];
        info->rdiag_min = smin[0];
        if (sbad[0]) info_event(info, CTQR_NONFINITE, -1);
        else if (first < n) info_event(info, CTQR_RANK_DEFICIENT, first);
    }
}

// out[k] = A(k, k) for k in [c0, c1)
template <typename T>
__global__ void diag_copy_kernel(int c0, int c1, const T *__restrict__ A, int64_t lda, T *__restrict__ out)
{
    const int k = c0 + (int)(blockIdx.x * blockDim.x + threadIdx.x);
    if (k < c1) out[k] = A[(int64_t)k * lda + k];
}

template <typename T>
__global__ void zero_kernel(T *__restrict__ p, int64_t count)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = T(0);
}

// RinvT block i = transpose of Rinv block i (each BIG x BIG, ld BIG)
template <typename T>
__global__ void block_transpose_kernel(const T *__restrict__ Rinv, T *__restrict__ RinvT, int z0)
{
    __shared__ T t[32][33];
    const int64_t base = (int64_t)(z0 + (int)blockIdx.z) * BIG * BIG;
    const int r0 = blockIdx.x * 32, c0 = blockIdx.y * 32;
    for (int k = threadIdx.y; k < 32; k += 8)
        t[k][threadIdx.x] = Rinv[base + (int64_t)(c0 + k) * BIG + r0 + threadIdx.x];
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += 8)
        RinvT[base + (int64_t)(r0 + k) * BIG + c0 + threadIdx.x] = t[threadIdx.x][k];
}

}  // namespace

// elements of the block inverses of R; the block transposes follow them, so a
// factor stores 2 * trinv_elems(n)
size_t trinv_elems(int n) { return (size_t)BIG * (size_t)ceil_div(n, BIG) * BIG; }
size_t trinv_tmp_elems() { return (size_t)(BIG / 2) * (BIG / 2); }

template <typename T>
ctqr_status trinv_blocks_range(int n, int c0, int c1, const T *R, int64_t ldr, T *Rinv, T *tmp, hipStream_t st)
{
    // Rinv holds the inverses, Rinv + trinv_elems(n) their block transposes;
    // this call fills the diagonal blocks whose columns start in [c0, c1)
    // (multiples of the block size) and reads R only inside them.
    const int64_t total = (int64_t)trinv_elems(n);
    c1 = std::min(c1, n);
    if (c0 >= c1) return CTQR_OK;
    const int64_t z0 = c0 / BIG, z1 = ceil_div(c1, BIG);
    const int64_t span = (z1 - z0) * BIG * BIG;
    LAUNCH_TRY(zero_kernel<T>, dim3((unsigned)std::min<int64_t>(ceil_div(span, 256), 8192)), dim3(256), 0, st,
               Rinv + z0 * BIG * BIG, span);
    LAUNCH_TRY(trinv_kernel<T>, dim3((unsigned)ceil_div(c1 - c0, BT), NQ), dim3(256), 0, st, n, R, ldr, Rinv,
               c0 / BT);
    // doubling inside every BIG block: [A B; 0 D] -> X12 = -inv(A) (B inv(D)).
    // The whole blocks of the range take each step as one batched launch over
    // the blocks, the product B inv(D) held in the block-transpose area at
    // X12's place (written by the transposes only at the end); a last,
    // partial block takes its steps one by one through tmp.
    const int64_t zf = std::min<int64_t>(z1, n / BIG);   // whole blocks: [z0, zf)
    if (zf > z0) {
        const int nbat = (int)(zf - z0);
        for (int s = BT; s < BIG; s *= 2) {
            for (int q = 0; q < BIG / (2 * s); ++q) {
                const int64_t g0 = z0 * BIG + 2LL * s * q, off = 2LL * s * q;
                const T *Bblk = R + (g0 + s) * ldr + g0;
                const T *Dinv = Rinv + (g0 + s) * BIG + off + s;
                const T *Ainv = Rinv + g0 * BIG + off;
                T *X12 = Rinv + (g0 + s) * BIG + off;
                T *Y = X12 + total;
                const int64_t bsr = (int64_t)BIG * ldr + BIG, bsi = (int64_t)BIG * BIG;
                ctqr_status e = gemm_nn_batched<T>(s, s, s, Bblk, ldr, bsr, Dinv, BIG, bsi, T(1), Y, BIG, bsi, nbat,
                                                   0, st);
                if (e) return e;
                e = gemm_nn_batched<T>(s, s, s, Ainv, BIG, bsi, Y, BIG, bsi, T(-1), X12, BIG, bsi, nbat, 0, st);
                if (e) return e;
            }
        }
    }
    const int64_t ldy = BIG / 2;
    for (int s = BT; s < BIG; s *= 2) {
        for (int g0 = (int)std::max<int64_t>(c0, zf * BIG); g0 < c1; g0 += 2 * s) {
            const int d = std::min(s, n - (g0 + s));
            if (d <= 0) continue;
            const int off = g0 % BIG;
            const T *Bblk = R + (int64_t)(g0 + s) * ldr + g0;               // s x d
            const T *Dinv = Rinv + (int64_t)(g0 + s) * BIG + off + s;         // d x d
            const T *Ainv = Rinv + (int64_t)g0 * BIG + off;                   // s x s
            T *X12 = Rinv + (int64_t)(g0 + s) * BIG + off;                    // s x d
            ctqr_status e = gemm_nn<T>(s, d, d, Bblk, ldr, 0, Dinv, BIG, T(1), tmp, ldy, nullptr, st, 0, 0);
            if (e) return e;
            e = gemm_nn<T>(s, d, s, Ainv, BIG, 0, tmp, ldy, T(-1), X12, BIG, nullptr, st, 0, 0);
            if (e) return e;
        }
    }
    LAUNCH_TRY(block_transpose_kernel<T>, dim3(BIG / 32, BIG / 32, (unsigned)(z1 - z0)), dim3(32, 8), 0, st,
               (const T *)Rinv, Rinv + total, (int)z0);
    return CTQR_OK;
}

template <typename T>
ctqr_status trinv_blocks(int n, const T *R, int64_t ldr, T *Rinv, T *tmp, ctqr_info *info, hipStream_t st)
{
    (void)info;
    return trinv_blocks_range<T>(n, 0, (int)(ceil_div(n, BIG) * BIG), R, ldr, Rinv, tmp, st);
}

template <typename T>
ctqr_status diag_copy(int c0, int c1, const T *A, int64_t lda, T *out, hipStream_t st)
{
    if (c1 <= c0) return CTQR_OK;
    LAUNCH_TRY(diag_copy_kernel<T>, dim3((unsigned)ceil_div(c1 - c0, 256)), dim3(256), 0, st, c0, c1, A, lda, out);
    return CTQR_OK;
}

template <typename T>
ctqr_status rdiag_check(int n, const T *R, int64_t ldr, double *scratch, ctqr_info *info,
                        hipStream_t st)
{
    (void)scratch;
    LAUNCH_TRY(rdiag_kernel<T>, dim3(1), dim3(1024), 0, st, n, R, ldr, info);
    return CTQR_OK;
}

// Block back substitution R X = C with the stored diagonal-block inverses
// (Section II-C, "System solving"), C overwritten.  Two orders with the same
// arithmetic per block:
//  - right-looking: after X_i, the rows above take its update at once,
//    C_{0:r0} -= R_{0:r0, i} X_i (products of r0 rows: few tiles early on);
//  - left-looking: before X_i, block row i takes the updates of every solved
//    block at once, C_i -= R_{i, i+1:} X_{i+1:} (a 2048-row product with a
//    long inner dimension, split over it, so every step fills the chip).
// Narrow right-hand sides (the 32-wide slice tile) use the left-looking order.
// Split-BF16 products for the off-diagonal blocks of a wide substitution
// (FP32 factor, at least one 128-wide slice tile, parts of R given): the
// refinement applies (R^T R)^-1 only to contract its error, which needs the
// accuracy of the factor itself (about 16 bits for a split-BF16 factor), not
// FP32's.  The diagonal-block products with the stored inverses stay FP32.
// R's off-diagonal blocks are split once (trsm_split_r) into the two layouts
// the products read:
//   nn: block column R_{0:r0, i} (i >= 1) as row-major high / low parts,
//       row stride BIG, at nn_off(i); the high part's r0 rows, then the low's.
//   tn: block row R_{i, i+1:} (i before the last) as column-major parts,
//       column stride BIG, columns padded to 128, at tn_off(i).
// The right-hand side X_i (Y_i) of each product is split per call into x.
namespace {
int64_t up128(int64_t v) { return ceil_div(v, 128) * 128; }
int64_t nn_off(int i) { return (int64_t)BIG * BIG * i * (i - 1); }
int64_t tn_off(int n, int i)
{
    int64_t off = 0;
    for (int j = 0; j < i; ++j) off += 2LL * BIG * up128(n - (int64_t)(j + 1) * BIG);
    return off;
}
}  // namespace

size_t trsm_rparts_elems(int64_t n)
{
    const int nblk = (int)ceil_div(n, BIG);
    return (size_t)(nn_off(nblk) + tn_off((int)n, std::max(0, nblk - 1)));
}

size_t trsm_xparts_elems(int S) { return (size_t)(2 * up128(S) * BIG); }

ctqr_status trsm_split_r(int n, const float *R, int64_t ldr, __bf16 *parts, hipStream_t st)
{
    const int nblk = (int)ceil_div(n, BIG);
    __bf16 *nn = parts, *tn = parts + nn_off(nblk);
    ctqr_status s;
    for (int i = 1; i < nblk; ++i) {
        const int r0 = i * BIG, bw = std::min(BIG, n - r0);
        __bf16 *hi = nn + nn_off(i);
        if ((s = bf16x3_split_rows(r0, bw, R + (int64_t)r0 * ldr, ldr, false, hi, hi + (int64_t)r0 * BIG, BIG, r0,
                                   st)))
            return s;
    }
    for (int i = 0; i + 1 < nblk; ++i) {
        const int r0 = i * BIG, rest = n - r0 - BIG;
        if ((s = bf16x3_split_vt(BIG, rest, R + (int64_t)(r0 + BIG) * ldr + r0, ldr, tn + tn_off(n, i),
                                 2 * (size_t)BIG * up128(rest), st, false)))
            return s;
    }
    return CTQR_OK;
}

template <typename T>
ctqr_status trsm_upper(int n, int S, const T *R, int64_t ldr, const T *Rinv, T *C, int64_t ldc,
                       T *X, int64_t ldx, T *part, size_t part_elems, const int *skip, hipStream_t st,
                       const TrsmParts *rp)
{
    const bool bf = sizeof(T) == 4 && rp && S >= TRSM_SPLIT_MIN_SLICES;
    const T *RinvT = Rinv + trinv_elems(n);
    const int nblk = (int)ceil_div(n, BIG);
    const bool left = S <= gemm_narrow_max();
    for (int i = nblk - 1; i >= 0; --i) {
        const int r0 = i * BIG, bw = min(BIG, n - r0);
        ctqr_status s;
        if (left && r0 + bw < n) {
            // C_i -= R_{i, i+1:} X_{i+1:}
            s = gemm_nn_split<T>(bw, S, n - r0 - bw, R + (int64_t)(r0 + bw) * ldr + r0, ldr, X + r0 + bw, ldx,
                                 T(-1), C + r0, ldc, part, part_elems, skip, st);
            if (s) return s;
        }
        // X_i = inv(R_ii) C_i = (inv(R_ii)^T)^T C_i  (split-K TN product)
        s = gemm_tn<T>(bw, S, bw, RinvT + (int64_t)r0 * BIG, BIG, 0, C + r0, ldc, 0, T(1), T(0), X + r0, ldx,
                       part, part_elems, skip, st, 0, 0, 1);
        if (s) return s;
        if (!left && r0 > 0) {
            // C_{0:r0} -= R_{0:r0, i} X_i
            if constexpr (sizeof(T) == 4) {
                if (bf) {
                    const __bf16 *ah = rp->r + nn_off(i), *al = ah + (int64_t)r0 * BIG;
                    const int cp = (int)up128(S);
                    __bf16 *xh = rp->x, *xl = rp->x + (int64_t)cp * BIG;
                    s = bf16x3_split_cols(bw, S, X + r0, ldx, xh, xl, BIG, cp, st, skip);
                    if (!s) s = gemm_nn_bf16x3_parts(r0, S, bw, -1.0f, C, ldc, ah, al, BIG, xh, xl, BIG, st, skip);
                    if (s) return s;
                    continue;
                }
            }
            s = gemm_nn<T>(r0, S, bw, R + (int64_t)r0 * ldr, ldr, 0, X + r0, ldx, T(-1), C, ldc, skip, st);
            if (s) return s;
        }
    }
    return CTQR_OK;
}

// Block forward substitution R^T Y = C, C overwritten; right-looking
// (C_{i+1:} -= R_{i, i+1:}^T Y_i after Y_i) or, for narrow right-hand
// sides, left-looking (C_i -= R_{0:r0, i}^T Y_{0:r0} before Y_i).
template <typename T>
ctqr_status trsm_upper_trans(int n, int S, const T *R, int64_t ldr, const T *Rinv, T *C, int64_t ldc,
                             T *Y, int64_t ldy, T *part, size_t part_elems, const int *skip,
                             hipStream_t st, const TrsmParts *rp)
{
    const bool bf = sizeof(T) == 4 && rp && S >= TRSM_SPLIT_MIN_SLICES;
    const int nblk = (int)ceil_div(n, BIG);
    const bool left = S <= gemm_narrow_max();
    for (int i = 0; i < nblk; ++i) {
        const int r0 = i * BIG, bw = min(BIG, n - r0);
        ctqr_status s;
        if (left && r0 > 0) {
            // C_i -= (R_{0:r0, i})^T Y_{0:r0}
            s = gemm_tn<T>(bw, S, r0, R + (int64_t)r0 * ldr, ldr, 0, Y, ldy, 0, T(-1), T(1), C + r0, ldc, part,
                           part_elems, skip, st);
            if (s) return s;
        }
        // Y_i = inv(R_ii)^T C_i
        s = gemm_tn<T>(bw, S, bw, Rinv + (int64_t)r0 * BIG, BIG, 0, C + r0, ldc, 0, T(1), T(0), Y + r0, ldy,
                       part, part_elems, skip, st, 0, 0, 2);
        if (s) return s;
        const int rest = n - r0 - bw;
        if (!left && rest > 0) {
            // C_{i+1:} -= (R_{i, i+1:})^T Y_i
            if constexpr (sizeof(T) == 4) {
                if (bf) {
                    const int nblk = (int)ceil_div(n, BIG);
                    const __bf16 *vt = rp->r + nn_off(nblk) + tn_off(n, i);
                    s = gemm_tn_bf16x3(rest, S, bw, vt, 2 * (size_t)BIG * up128(rest), Y + r0, ldy, 0, -1.0f, 1.0f,
                                       C + r0 + bw, ldc, part, part_elems, skip, st, 0);
                    if (s) return s;
                    continue;
                }
            }
            s = gemm_tn<T>(rest, S, bw, R + (int64_t)(r0 + bw) * ldr + r0, ldr, 0, Y + r0, ldy, 0,
                           T(-1), T(1), C + r0 + bw, ldc, part, part_elems, skip, st);
            if (s) return s;
        }
    }
    return CTQR_OK;
}

// Column-block ranges of the two substitutions, for a factor whose columns
// are not all addressable at once (R: column k at R + k ldr for the columns
// of the range only).  trsm_upper_cols runs the right-looking steps of the
// diagonal blocks starting in [c_lo, c_hi), last block first: each step reads
// only its own column block of R, so the ranges are taken from the last to
// the first.  trsm_upper_trans_cols runs the left-looking steps of the blocks
// in the range, first block first, also reading only column block i.
template <typename T>
ctqr_status trsm_upper_cols(int n, int S, const T *R, int64_t ldr, const T *Rinv, T *C, int64_t ldc, T *X,
                            int64_t ldx, int c_lo, int c_hi, T *part, size_t part_elems, const int *skip,
                            hipStream_t st)
{
    const T *RinvT = Rinv + trinv_elems(n);
    for (int r0 = (int)(ceil_div(std::min(c_hi, n), BIG) - 1) * BIG; r0 >= c_lo; r0 -= BIG) {
        const int bw = min(BIG, n - r0);
        ctqr_status s = gemm_tn<T>(bw, S, bw, RinvT + (int64_t)r0 * BIG, BIG, 0, C + r0, ldc, 0, T(1), T(0),
                                   X + r0, ldx, part, part_elems, skip, st, 0, 0, 1);
        if (s) return s;
        if (r0 > 0) {
            s = gemm_nn<T>(r0, S, bw, R + (int64_t)r0 * ldr, ldr, 0, X + r0, ldx, T(-1), C, ldc, skip, st);
            if (s) return s;
        }
    }
    return CTQR_OK;
}

template <typename T>
ctqr_status trsm_upper_trans_cols(int n, int S, const T *R, int64_t ldr, const T *Rinv, T *C, int64_t ldc, T *Y,
                                  int64_t ldy, int c_lo, int c_hi, T *part, size_t part_elems, const int *skip,
                                  hipStream_t st)
{
    for (int r0 = c_lo; r0 < std::min(c_hi, n); r0 += BIG) {
        const int bw = min(BIG, n - r0);
        ctqr_status s;
        if (r0 > 0) {
            s = gemm_tn<T>(bw, S, r0, R + (int64_t)r0 * ldr, ldr, 0, Y, ldy, 0, T(-1), T(1), C + r0, ldc, part,
                           part_elems, skip, st);
            if (s) return s;
        }
        s = gemm_tn<T>(bw, S, bw, Rinv + (int64_t)r0 * BIG, BIG, 0, C + r0, ldc, 0, T(1), T(0), Y + r0, ldy,
                       part, part_elems, skip, st, 0, 0, 2);
        if (s) return s;
    }
    return CTQR_OK;
}

#define INST(T)                                                                                        \
    template ctqr_status trinv_blocks<T>(int, const T *, int64_t, T *, T *, ctqr_info *, hipStream_t);  \
    template ctqr_status trinv_blocks_range<T>(int, int, int, const T *, int64_t, T *, T *, hipStream_t); \
    template ctqr_status rdiag_check<T>(int, const T *, int64_t, double *, ctqr_info *, hipStream_t);   \
    template ctqr_status diag_copy<T>(int, int, const T *, int64_t, T *, hipStream_t);                  \
    template ctqr_status trsm_upper<T>(int, int, const T *, int64_t, const T *, T *, int64_t, T *,       \
                                       int64_t, T *, size_t, const int *, hipStream_t, const TrsmParts *); \
    template ctqr_status trsm_upper_trans<T>(int, int, const T *, int64_t, const T *, T *, int64_t,     \
                                             T *, int64_t, T *, size_t, const int *, hipStream_t,       \
                                             const TrsmParts *);                                         \
    template ctqr_status trsm_upper_cols<T>(int, int, const T *, int64_t, const T *, T *, int64_t, T *,  \
                                            int64_t, int, int, T *, size_t, const int *, hipStream_t);  \
    template ctqr_status trsm_upper_trans_cols<T>(int, int, const T *, int64_t, const T *, T *, int64_t, \
                                                  T *, int64_t, int, int, T *, size_t, const int *,    \
                                                  hipStream_t);
INST(float)
INST(double)
