// Block triangular solves with the R factor (Section II-C, "System solving":
// the block-row backward substitution of Trsm_lunn / Gemm_nn_mo tasks).
//
//   trsm_upper:        R X = C, block rows from the bottom:
//                      X_i = R_ii^-1 C_i;  C_{0:i} -= R_{0:i, i} X_i
//   trsm_upper_trans:  R^T Y = C, block rows from the top (used by the
//                      refinement's semi-normal equations):
//                      Y_i = R_ii^-T C_i;  C_{i+1:} -= R_{i, i+1:}^T Y_i
//
// The diagonal 64 x 64 blocks are inverted once (trinv_blocks, one workgroup
// per block, FP64 arithmetic), so both the diagonal solve and the off-diagonal
// update are MFMA products; only the 64-row block chain is sequential.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int BT = TRSM_BT;

// Inverse of each BT x BT upper-triangular diagonal block of R.  Thread j
// computes column j of the inverse by back substitution on e_j.  Rinv holds
// the inverse blocks (BT x n, block i at columns i*BT), RinvT their
// transposes.  Zero or non-finite diagonals are reported (rank deficiency is
// diagnosed separately by rdiag_check).
template <typename T>
__global__ __launch_bounds__(BT)
void trinv_kernel(int n, const T *__restrict__ R, int64_t ldr, T *__restrict__ Rinv,
                  T *__restrict__ RinvT)
{
    __shared__ double Rs[BT][BT + 1];
    __shared__ double Xs[BT][BT + 1];
    const int blk = blockIdx.x, j = threadIdx.x;
    const int base = blk * BT;
    const int nbk = min(BT, n - base);
    for (int c = 0; c < BT; ++c) {
        double v = 0.0;
        if (j < nbk && c < nbk) v = (double)R[(int64_t)(base + c) * ldr + base + j];
        Rs[j][c] = v;   // Rs[row][col]
    }
    __syncthreads();
    // column j of inv(R_bb)
    for (int i = BT - 1; i >= 0; --i) {
        double x = 0.0;
        if (j < nbk && i < nbk && i <= j) {
            double s = (i == j) ? 1.0 : 0.0;
            for (int k = i + 1; k <= j; ++k) s -= Rs[i][k] * Xs[k][j];
            x = s / Rs[i][i];
        }
        Xs[i][j] = x;
    }
    __syncthreads();
    for (int i = 0; i < BT; ++i) {
        // Rinv block: column j contiguous in i; RinvT block: (i, j) -> (j, i)
        Rinv[(int64_t)(base + j) * BT + i] = (T)Xs[i][j];
        RinvT[(int64_t)(base + i) * BT + j] = (T)Xs[i][j];
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

}  // namespace

template <typename T>
ctqr_status trinv_blocks(int n, const T *R, int64_t ldr, T *Rinv, T *RinvT, ctqr_info *info,
                         hipStream_t st)
{
    (void)info;
    LAUNCH_TRY(trinv_kernel<T>, dim3((unsigned)ceil_div(n, BT)), dim3(BT), 0, st, n, R, ldr, Rinv, RinvT);
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

template <typename T>
ctqr_status trsm_upper(int n, int S, const T *R, int64_t ldr, const T *RinvT, T *C, int64_t ldc,
                       T *X, int64_t ldx, T *part, size_t part_elems, const int *skip, hipStream_t st)
{
    const int nblk = (int)ceil_div(n, BT);
    for (int i = nblk - 1; i >= 0; --i) {
        const int r0 = i * BT, bw = min(BT, n - r0);
        // X_i = inv(R_ii) C_i  ==  (RinvT_i)^T C_i
        ctqr_status s = gemm_tn<T>(bw, S, bw, RinvT + (int64_t)r0 * BT, BT, 0, C + r0, ldc, 0,
                                   T(1), T(0), X + r0, ldx, part, part_elems, skip, st);
        if (s) return s;
        if (r0 > 0) {
            // C_{0:r0} -= R_{0:r0, i} X_i
            s = gemm_nn<T>(r0, S, bw, R + (int64_t)r0 * ldr, ldr, 0, X + r0, ldx, T(-1), C, ldc,
                           skip, st);
            if (s) return s;
        }
    }
    return CTQR_OK;
}

template <typename T>
ctqr_status trsm_upper_trans(int n, int S, const T *R, int64_t ldr, const T *Rinv, T *C, int64_t ldc,
                             T *Y, int64_t ldy, T *part, size_t part_elems, const int *skip,
                             hipStream_t st)
{
    const int nblk = (int)ceil_div(n, BT);
    for (int i = 0; i < nblk; ++i) {
        const int r0 = i * BT, bw = min(BT, n - r0);
        // Y_i = inv(R_ii)^T C_i
        ctqr_status s = gemm_tn<T>(bw, S, bw, Rinv + (int64_t)r0 * BT, BT, 0, C + r0, ldc, 0,
                                   T(1), T(0), Y + r0, ldy, part, part_elems, skip, st);
        if (s) return s;
        const int rest = n - r0 - bw;
        if (rest > 0) {
            // C_{i+1:} -= (R_{i, i+1:})^T Y_i
            s = gemm_tn<T>(rest, S, bw, R + (int64_t)(r0 + bw) * ldr + r0, ldr, 0, Y + r0, ldy, 0,
                           T(-1), T(1), C + r0 + bw, ldc, part, part_elems, skip, st);
            if (s) return s;
        }
    }
    return CTQR_OK;
}

#define INST(T)                                                                                   \
    template ctqr_status trinv_blocks<T>(int, const T *, int64_t, T *, T *, ctqr_info *, hipStream_t); \
    template ctqr_status rdiag_check<T>(int, const T *, int64_t, double *, ctqr_info *, hipStream_t);  \
    template ctqr_status trsm_upper<T>(int, int, const T *, int64_t, const T *, T *, int64_t, T *,      \
                                       int64_t, T *, size_t, const int *, hipStream_t);                \
    template ctqr_status trsm_upper_trans<T>(int, int, const T *, int64_t, const T *, T *, int64_t,    \
                                             T *, int64_t, T *, size_t, const int *, hipStream_t);
INST(float)
INST(double)
