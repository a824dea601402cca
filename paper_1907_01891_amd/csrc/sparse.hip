// FP64 sparse products with the Siddon matrix, layout conversions and the
// refinement bookkeeping kernels.
//
// The refinement (corrected semi-normal equations) needs r = B - A X and
// s = A^T r in FP64 with the exact sparse A.  Both are gathers: rows of the
// CSR for A X, rows of the CSC (= columns of A) for A^T r, with the slice
// vectors stored row-major (slice index fastest) so that the lanes of a
// workgroup read one contiguous row of X per nonzero.
#include <cmath>

#include "common.h"
#include "kernels.h"

namespace {

// Row visited in place of row i when the rows are the pixels of a tside x
// tside image (row iy * tside + ix, tside a multiple of 16): the image in
// 16 x 16 tiles, tile rows in order.  Neighbouring pixels are crossed by the
// same rays, so the rows gathered for one tile are shared in the L2; the
// results do not depend on the order.
__device__ inline int64_t pixel_tile_row(int64_t i, int tside)
{
    if (tside <= 0) return i;
    const int64_t t = i / 256, w = i % 256, tpr = tside / 16;
    return ((t / tpr) * 16 + w / 16) * tside + (t % tpr) * 16 + w % 16;
}

// y[i, s] = alpha * sum_k val[k] x[idx[k], s] + beta * y_in[i, s]
// Wide form (S > 64): SW = min(256, S rounded up to 64) threads per row, one
// slice per thread.
__global__ __launch_bounds__(256)
void spmm_rm_kernel(int64_t rows, int S, int SW, const int64_t *__restrict__ ptr,
                    const int32_t *__restrict__ idx, const double *__restrict__ val, double alpha,
                    const double *__restrict__ x, double beta, const double *__restrict__ y_in,
                    double *__restrict__ y, const int *skip, int tside)
{
    if (skip && *skip) return;
    const int rpb = 256 / SW;
    // consecutive rows (neighbouring rays, which cross neighbouring pixels)
    // go to the same XCD so the gathered rows of x are shared in its L2
    unsigned blk = blockIdx.x;
    const unsigned per = gridDim.x / 8;
    if (blk < per * 8) blk = (blk % 8) * per + blk / 8;
    const int64_t i0 = (int64_t)blk * rpb + threadIdx.x / SW;
    const int lane = threadIdx.x % SW;
    if (i0 >= rows) return;
    const int64_t i = pixel_tile_row(i0, tside);
    const int64_t b = ptr[i], e = ptr[i + 1];
    for (int s0 = 0; s0 < S; s0 += SW) {
        const int s = s0 + lane;
        if (s >= S) break;
        double acc = 0.0;
#pragma unroll 4
        for (int64_t k = b; k < e; ++k) acc += val[k] * x[(int64_t)idx[k] * S + s];
        double out = alpha * acc;
        if (beta != 0.0) out += beta * y_in[i * S + s];
        y[i * S + s] = out;
    }
}

// Wide rows (S > 192, one row per workgroup, slice s0 + 256 p in thread
// s0): the row's indices and values staged in LDS 256 at a time, so each
// thread keeps sixteen gathers of x in flight instead of waiting on an index
// load before each one.  Same products in the same order as spmm_rm_kernel.
template <int MAXP>
__global__ __launch_bounds__(256)
void spmm_rm_staged_kernel(int64_t rows, int S, const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                           const double *__restrict__ val, double alpha, const double *__restrict__ x, double beta,
                           const double *__restrict__ y_in, double *__restrict__ y, const int *skip, int tside)
{
    if (skip && *skip) return;
    __shared__ int32_t si[256];
    __shared__ double sv[256];
    unsigned blk = blockIdx.x;
    const unsigned per = gridDim.x / 8;
    if (blk < per * 8) blk = (blk % 8) * per + blk / 8;
    if ((int64_t)blk >= rows) return;
    const int64_t i = pixel_tile_row(blk, tside);
    const int tid = threadIdx.x;
    const int P = (S + 255) / 256;
    const int64_t b = ptr[i], e = ptr[i + 1];
    double acc[MAXP];
#pragma unroll
    for (int p = 0; p < MAXP; ++p) acc[p] = 0.0;
    for (int64_t c0 = b; c0 < e; c0 += 256) {
        const int n = (int)min((int64_t)256, e - c0);
        __syncthreads();
        if (tid < n) {
            si[tid] = idx[c0 + tid];
            sv[tid] = val[c0 + tid];
        }
        __syncthreads();
#pragma unroll
        for (int p = 0; p < MAXP; ++p) {
            const int sl = 256 * p + tid;
            if (p < P && sl < S) {
                double a = acc[p];
#pragma unroll 16
                for (int k = 0; k < n; ++k) a += sv[k] * x[(int64_t)si[k] * S + sl];
                acc[p] = a;
            }
        }
    }
#pragma unroll
    for (int p = 0; p < MAXP; ++p) {
        const int sl = 256 * p + tid;
        if (p < P && sl < S) {
            double out = alpha * acc[p];
            if (beta != 0.0) out += beta * y_in[i * S + sl];
            y[i * S + sl] = out;
        }
    }
}

// Narrow form (S <= 64): one wave per row, its lanes split into 64 / SP
// groups of SP slices (SP = S rounded up to a power of two).  Group g sums the
// row's nonzeros g, g + G, g + 2G, ... in order; the groups' sums are then
// combined by a fixed butterfly, so the result does not depend on timing.
template <int SP>
__global__ __launch_bounds__(256)
void spmm_rm_narrow_kernel(int64_t rows, int S, const int64_t *__restrict__ ptr,
                           const int32_t *__restrict__ idx, const double *__restrict__ val, double alpha,
                           const double *__restrict__ x, double beta, const double *__restrict__ y_in,
                           double *__restrict__ y, const int *skip)
{
    if (skip && *skip) return;
    constexpr int G = CTQR_WAVE / SP;
    unsigned blk = blockIdx.x;
    const unsigned per = gridDim.x / 8;
    if (blk < per * 8) blk = (blk % 8) * per + blk / 8;
    const int64_t i = (int64_t)blk * 4 + threadIdx.x / CTQR_WAVE;
    const int lane = threadIdx.x % CTQR_WAVE;
    const int g = lane / SP, s = lane % SP;
    if (i >= rows) return;   // whole waves leave together
    const int64_t b = ptr[i], e = ptr[i + 1];
    double acc = 0.0;
    if (s < S) {
#pragma unroll 4
        for (int64_t k = b + g; k < e; k += G) acc += val[k] * x[(int64_t)idx[k] * S + s];
    }
#pragma unroll
    for (int off = SP; off < CTQR_WAVE; off <<= 1) acc += __shfl_xor(acc, off);
    if (g == 0 && s < S) {
        double out = alpha * acc;
        if (beta != 0.0) out += beta * y_in[i * S + s];
        y[i * S + s] = out;
    }
}

// Column-major variant for the public helper: thread per (row, slice).
__global__ void spmm_cm_kernel(int64_t rows, int S, const int64_t *__restrict__ ptr,
                               const int32_t *__restrict__ idx, const double *__restrict__ val,
                               double alpha, const double *__restrict__ X, int64_t ldx, double beta,
                               double *__restrict__ Y, int64_t ldy)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int s = blockIdx.y;
    if (i >= rows) return;
    double acc = 0.0;
    for (int64_t k = ptr[i]; k < ptr[i + 1]; ++k) acc += val[k] * X[(int64_t)s * ldx + idx[k]];
    double *o = Y + (int64_t)s * ldy + i;
    *o = beta == 0.0 ? alpha * acc : alpha * acc + beta * *o;
}

// Tiled transposes between column-major (rows x S, ld) and row-major (rows x S).
template <typename TD, typename TSRC>
__global__ void cm_to_rm_kernel(int64_t rows, int S, const TSRC *__restrict__ src, int64_t lds,
                                TD *__restrict__ dst, const int *skip)
{
    if (skip && *skip) return;
    __shared__ double t[32][33];
    const int64_t r0 = (int64_t)blockIdx.x * 32;
    const int s0 = blockIdx.y * 32;
    for (int k = threadIdx.y; k < 32; k += 8) {
        int64_t r = r0 + threadIdx.x;
        int s = s0 + k;
        t[k][threadIdx.x] = (r < rows && s < S) ? (double)src[(int64_t)s * lds + r] : 0.0;
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += 8) {
        int64_t r = r0 + k;
        int s = s0 + threadIdx.x;
        if (r < rows && s < S) dst[r * S + s] = (TD)t[threadIdx.x][k];
    }
}

template <typename TD, typename TSRC>
__global__ void rm_to_cm_kernel(int64_t rows, int S, int ss, const TSRC *__restrict__ src,
                                TD *__restrict__ dst, int64_t ldd, const int *skip)
{
    // the first S of the ss values of each source row
    if (skip && *skip) return;
    __shared__ double t[32][33];
    const int64_t r0 = (int64_t)blockIdx.x * 32;
    const int s0 = blockIdx.y * 32;
    for (int k = threadIdx.y; k < 32; k += 8) {
        int64_t r = r0 + k;
        int s = s0 + threadIdx.x;
        t[k][threadIdx.x] = (r < rows && s < S) ? (double)src[r * ss + s] : 0.0;
    }
    __syncthreads();
    for (int k = threadIdx.y; k < 32; k += 8) {
        int64_t r = r0 + threadIdx.x;
        int s = s0 + k;
        if (r < rows && s < S) dst[(int64_t)s * ldd + r] = (TD)t[threadIdx.x][k];
    }
}

template <typename TD, typename TSRC>
__global__ void copy_cm_kernel(int64_t rows, int S, const TSRC *__restrict__ src, int64_t lds,
                               TD *__restrict__ dst, int64_t ldd)
{
    const int s = blockIdx.y;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x)
        dst[(int64_t)s * ldd + r] = (TD)src[(int64_t)s * lds + r];
}

__global__ void fill_u32_kernel(unsigned *p, int64_t n, unsigned v)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

__global__ void fill_f64_kernel(double *p, int64_t n, double v)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = v;
}

__global__ void info_reset_kernel(ctqr_info *info)
{
    info->status = 0;
    info->first_bad_col = -1;
    info->iters = 0;
    info->x_iters = 0;
    info->max_rel_update = 0.0;
    info->rdiag_max = 0.0;
    info->rdiag_min = 0.0;
    info->nnz = 0;
    info->contraction = 0.0;
}

// Non-negative doubles order like their bit patterns; NaN maps to all ones.
__device__ inline unsigned long long order_bits(double v)
{
    v = fabs(v);
    return v == v ? (unsigned long long)__double_as_longlong(v) : ~0ull;
}

// x += d; xs (when given) receives x before the update, the iterate whose
// error this update estimates.
template <typename TD>
__global__ void refine_update_kernel(int64_t n, int S, double *__restrict__ x, const TD *__restrict__ d,
                                     int64_t ldd, unsigned long long *dmax, unsigned long long *xmax,
                                     double *__restrict__ xs, const int *skip)
{
    if (skip && *skip) return;
    __shared__ double t[32][33];
    __shared__ unsigned long long md[8][32], mx[8][32];
    const int s0 = blockIdx.y * 32;
    const int s = s0 + threadIdx.x;
    unsigned long long dm = 0, xm = 0;
    // 32-row tiles, strided over the grid: few blocks, so few atomics
    for (int64_t r0 = (int64_t)blockIdx.x * 32; r0 < n; r0 += (int64_t)gridDim.x * 32) {
        __syncthreads();
        for (int k = threadIdx.y; k < 32; k += 8) {
            int64_t r = r0 + threadIdx.x;
            int sk = s0 + k;
            t[k][threadIdx.x] = (r < n && sk < S) ? (double)d[(int64_t)sk * ldd + r] : 0.0;
        }
        __syncthreads();
        for (int k = threadIdx.y; k < 32; k += 8) {
            int64_t r = r0 + k;
            if (r < n && s < S) {
                double dv = t[threadIdx.x][k];
                const double xo = x[r * S + s];
                if (xs) xs[r * S + s] = xo;
                double xv = xo + dv;
                x[r * S + s] = xv;
                unsigned long long a = order_bits(dv), b = order_bits(xv);
                dm = a > dm ? a : dm;
                xm = b > xm ? b : xm;
            }
        }
    }
    md[threadIdx.y][threadIdx.x] = dm;
    mx[threadIdx.y][threadIdx.x] = xm;
    __syncthreads();
    if (threadIdx.y == 0 && s < S) {
        for (int k = 1; k < 8; ++k) {
            dm = md[k][threadIdx.x] > dm ? md[k][threadIdx.x] : dm;
            xm = mx[k][threadIdx.x] > xm ? mx[k][threadIdx.x] : xm;
        }
        atomicMax(&dmax[s], dm);
        atomicMax(&xmax[s], xm);
    }
}

// smax[s] = max over rows of |x[r, s]| (row-major rows x S; bit patterns,
// atomic max).  Block: 4 row groups x 64 slices.
__global__ __launch_bounds__(256)
void slice_absmax_kernel(int64_t rows, int S, const double *__restrict__ x, unsigned long long *smax,
                         const int *skip)
{
    if (skip && *skip) return;
    __shared__ unsigned long long red[4][64];
    const int lane = threadIdx.x % 64, grp = threadIdx.x / 64;
    const int s = blockIdx.y * 64 + lane;
    unsigned long long m = 0;
    if (s < S)
        for (int64_t r = (int64_t)blockIdx.x * 4 + grp; r < rows; r += (int64_t)gridDim.x * 4) {
            const unsigned long long b = order_bits(x[r * S + s]);
            m = b > m ? b : m;
        }
    red[grp][lane] = m;
    __syncthreads();
    if (grp == 0 && s < S) {
        for (int k = 1; k < 4; ++k) m = red[k][lane] > m ? red[k][lane] : m;
        atomicMax(&smax[s], m);
    }
}

// Decide convergence after refinement iteration `it` (0-based) and reset the
// per-slice maxima for the next one.  The refinement has converged when
// rel = max_s ||d_s||_inf / ||x_s||_inf <= tol.  It ends without converging
// (CTQR_NOT_CONVERGED) after stall_limit consecutive updates that are no
// smaller than 0.9x the previous one, or after max_iters.
// Which iterate is best is judged by the normal-equation residual
// s = A^T (b - A x) of the iterate before this iteration's update,
// g = max_s ||s_s||_inf / ||s_s^(0)||_inf: s = A^T A e for the error e of that
// iterate, whatever the quality of the preconditioner (the update itself
// estimates e only when (R^T R)^-1 A^T A is close to I).
// hist: [0] previous rel, [1] consecutive non-contracting updates, [2] the
// smallest g so far, [3] 1 once [2] is set, [4] 1 if this iteration set a new
// smallest g (the iterate before this update is the best one so far;
// refine_keep copies it), [5] the iteration that set [2], [6] the first rel,
// [7] the rel of the iteration that set [2].
__global__ __launch_bounds__(256)
void refine_check_kernel(int S, unsigned long long *dmax, unsigned long long *xmax, unsigned long long *smax,
                         double *s0, double tol, int it, int max_iters, int stall_limit, double *hist, int *done,
                         ctqr_info *info)
{
    if (*done) {
        if (threadIdx.x == 0) hist[4] = 0.0;
        return;
    }
    __shared__ double red[256];
    double worst = 0.0;
    bool bad = false;
    for (int s = threadIdx.x; s < S; s += 256) {
        unsigned long long a = dmax[s], b = xmax[s];
        if (a == ~0ull || b == ~0ull) { bad = true; continue; }
        double dv = __longlong_as_double((long long)a), xv = __longlong_as_double((long long)b);
        double rel = xv > 0.0 ? dv / xv : (dv > 0.0 ? INFINITY : 0.0);
        worst = fmax(worst, rel);
    }
    // normal-equation residual of this iteration's starting iterate, relative
    // to the first iteration's, per slice (zero slices count as 0)
    __shared__ double gred[256];
    double gw = 0.0;
    for (int s = threadIdx.x; s < S; s += 256) {
        unsigned long long a = smax[s];
        if (a == ~0ull) { bad = true; continue; }
        const double sv = __longlong_as_double((long long)a);
        if (it == 0) s0[s] = sv;
        const double b = s0[s];
        gw = fmax(gw, b > 0.0 ? sv / b : 0.0);
    }
    red[threadIdx.x] = bad ? INFINITY : worst;
    gred[threadIdx.x] = gw;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) {
            red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k]);
            gred[threadIdx.x] = fmax(gred[threadIdx.x], gred[threadIdx.x + k]);
        }
        __syncthreads();
    }
    for (int s = threadIdx.x; s < S; s += 256) {
        dmax[s] = 0;
        xmax[s] = 0;
        smax[s] = 0;
    }
    if (threadIdx.x == 0) {
        double rel = red[0];
        const double g = gred[0];
        info->iters = it + 1;
        info->x_iters = it + 1;
        info->max_rel_update = rel;
        if (it == 0) hist[6] = rel;
        info->contraction = (it > 0 && hist[6] > 0.0 && rel <= 1e300) ? pow(rel / hist[6], 1.0 / it) : 0.0;
        const bool better = rel <= 1e300 && (hist[3] == 0.0 || g < hist[2]);
        hist[4] = better ? 1.0 : 0.0;
        if (better) {
            hist[2] = g;
            hist[3] = 1.0;
            hist[5] = it;
            hist[7] = rel;
        }
        if (!(rel <= 1e300)) {
            info_event(info, CTQR_NONFINITE, -1);
            *done = 1;
        } else if (rel <= tol) {
            *done = 1;
        } else {
            double prev = hist[0];
            int stalls = (it > 0 && rel > 0.9 * prev) ? (int)hist[1] + 1 : 0;
            hist[0] = rel;
            hist[1] = stalls;
            if (stalls >= stall_limit || it + 1 >= max_iters) {
                info_event(info, CTQR_NOT_CONVERGED, -1);
                *done = 1;
            }
        }
    }
}

// xbest = xs when the last check found a new smallest update (hist[4]).
__global__ void refine_keep_kernel(int64_t count, const double *__restrict__ xs, double *__restrict__ xbest,
                                   const double *hist)
{
    if (hist[4] == 0.0) return;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        xbest[e] = xs[e];
}

// After a refinement that did not converge: x = xbest, the iterate with the
// smallest normal-equation residual, unless that was the last iteration's
// starting iterate (the residual was still falling, so the last iterate is
// kept).  The info then reports that iterate: x_iters updates,
// max_rel_update the update computed from it.
__global__ void refine_select_kernel(int64_t count, double *__restrict__ x, const double *__restrict__ xbest,
                                     const double *hist, ctqr_info *info)
{
    if (info->status != CTQR_NOT_CONVERGED || hist[3] == 0.0) return;
    const int best = (int)hist[5];
    if (best >= info->iters - 1) return;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < count;
         e += (int64_t)gridDim.x * blockDim.x)
        x[e] = xbest[e];
    __syncthreads();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        info->x_iters = best;
        info->max_rel_update = hist[7];
    }
}

}  // namespace

int pixel_tile_side(int64_t n)
{
    const int64_t side = (int64_t)std::llround(std::sqrt((double)n));
    return side * side == n && side % 16 == 0 ? (int)side : 0;
}

ctqr_status spmm_rowmajor(int64_t rows, int S, const int64_t *ptr, const int32_t *idx,
                          const double *val, double alpha, const double *x, double beta,
                          const double *y_in, double *y, const int *skip, hipStream_t st, int tside)
{
    if (rows <= 0 || S <= 0) return CTQR_OK;
    if (tside > 0 && (tside % 16 != 0 || (int64_t)tside * tside != rows)) return CTQR_EINVAL;
    if (S <= CTQR_WAVE) {
        dim3 grid((unsigned)ceil_div(rows, 4));
#define CTQR_SPMM_NARROW(SPV)                                                                       \
    LAUNCH_TRY(spmm_rm_narrow_kernel<SPV>, grid, dim3(256), 0, st, rows, S, ptr, idx, val, alpha, x, \
               beta, y_in, y, skip)
        if (S == 1) CTQR_SPMM_NARROW(1);
        else if (S == 2) CTQR_SPMM_NARROW(2);
        else if (S <= 4) CTQR_SPMM_NARROW(4);
        else if (S <= 8) CTQR_SPMM_NARROW(8);
        else if (S <= 16) CTQR_SPMM_NARROW(16);
        else if (S <= 32) CTQR_SPMM_NARROW(32);
        else CTQR_SPMM_NARROW(64);
#undef CTQR_SPMM_NARROW
        return CTQR_OK;
    }
    if (S > 192 && S <= 2048) {
#define CTQR_SPMM_STAGED(P)                                                                                    \
    LAUNCH_TRY(spmm_rm_staged_kernel<P>, dim3((unsigned)rows), dim3(256), 0, st, rows, S, ptr, idx, val, alpha, x, \
               beta, y_in, y, skip, tside)
        if (S <= 256) CTQR_SPMM_STAGED(1);
        else if (S <= 512) CTQR_SPMM_STAGED(2);
        else if (S <= 1024) CTQR_SPMM_STAGED(4);
        else CTQR_SPMM_STAGED(8);
#undef CTQR_SPMM_STAGED
        return CTQR_OK;
    }
    int SW = (int)std::min<int64_t>(256, ceil_div(S, 64) * 64);
    int rpb = 256 / SW;
    LAUNCH_TRY(spmm_rm_kernel, dim3((unsigned)ceil_div(rows, rpb)), dim3(256), 0, st, rows, S, SW, ptr,
               idx, val, alpha, x, beta, y_in, y, skip, tside);
    return CTQR_OK;
}

ctqr_status spmm_colmajor(int64_t rows, int64_t cols, int S, const int64_t *ptr, const int32_t *idx,
                          const double *val, double alpha, const double *X, int64_t ldx,
                          double beta, double *Y, int64_t ldy, hipStream_t st)
{
    (void)cols;
    if (rows <= 0 || S <= 0) return CTQR_OK;
    LAUNCH_TRY(spmm_cm_kernel, dim3((unsigned)ceil_div(rows, 256), (unsigned)S), dim3(256), 0, st, rows,
               S, ptr, idx, val, alpha, X, ldx, beta, Y, ldy);
    return CTQR_OK;
}

template <typename TD, typename TSRC>
ctqr_status cm_to_rm(int64_t rows, int S, const TSRC *src, int64_t lds, TD *dst, const int *skip,
                     hipStream_t st)
{
    if (rows <= 0 || S <= 0) return CTQR_OK;
    LAUNCH_TRY((cm_to_rm_kernel<TD, TSRC>), dim3((unsigned)ceil_div(rows, 32), (unsigned)ceil_div(S, 32)),
               dim3(32, 8), 0, st, rows, S, src, lds, dst, skip);
    return CTQR_OK;
}

template <typename TD, typename TSRC>
ctqr_status rm_to_cm(int64_t rows, int S, const TSRC *src, TD *dst, int64_t ldd, const int *skip,
                     hipStream_t st)
{
    if (rows <= 0 || S <= 0) return CTQR_OK;
    LAUNCH_TRY((rm_to_cm_kernel<TD, TSRC>), dim3((unsigned)ceil_div(rows, 32), (unsigned)ceil_div(S, 32)),
               dim3(32, 8), 0, st, rows, S, S, src, dst, ldd, skip);
    return CTQR_OK;
}

ctqr_status rm_to_cm_sub(int64_t rows, int ss, int S, const double *src, double *dst, int64_t ldd,
                         hipStream_t st)
{
    if (rows <= 0 || S <= 0) return CTQR_OK;
    LAUNCH_TRY((rm_to_cm_kernel<double, double>), dim3((unsigned)ceil_div(rows, 32), (unsigned)ceil_div(S, 32)),
               dim3(32, 8), 0, st, rows, S, ss, src, dst, ldd, nullptr);
    return CTQR_OK;
}

template <typename TD, typename TSRC>
ctqr_status copy_cm(int64_t rows, int S, const TSRC *src, int64_t lds, TD *dst, int64_t ldd,
                    hipStream_t st)
{
    if (rows <= 0 || S <= 0) return CTQR_OK;
    unsigned gx = (unsigned)std::min<int64_t>(ceil_div(rows, 256), 4096);
    LAUNCH_TRY((copy_cm_kernel<TD, TSRC>), dim3(gx, (unsigned)S), dim3(256), 0, st, rows, S, src, lds,
               dst, ldd);
    return CTQR_OK;
}

ctqr_status fill_u32(unsigned *p, int64_t n, unsigned v, hipStream_t st)
{
    if (n <= 0) return CTQR_OK;
    unsigned g = (unsigned)std::min<int64_t>(ceil_div(n, 256), 4096);
    LAUNCH_TRY(fill_u32_kernel, dim3(g), dim3(256), 0, st, p, n, v);
    return CTQR_OK;
}

ctqr_status fill_f64(double *p, int64_t n, double v, hipStream_t st)
{
    if (n <= 0) return CTQR_OK;
    unsigned g = (unsigned)std::min<int64_t>(ceil_div(n, 256), 4096);
    LAUNCH_TRY(fill_f64_kernel, dim3(g), dim3(256), 0, st, p, n, v);
    return CTQR_OK;
}

ctqr_status info_reset(ctqr_info *info, hipStream_t st)
{
    LAUNCH_TRY(info_reset_kernel, dim3(1), dim3(1), 0, st, info);
    return CTQR_OK;
}

template <typename TD>
ctqr_status refine_update(int64_t n, int S, double *x, const TD *d, int64_t ldd,
                          unsigned long long *dmax, unsigned long long *xmax, double *xs, const int *skip,
                          hipStream_t st)
{
    LAUNCH_TRY(refine_update_kernel<TD>, dim3((unsigned)std::min<int64_t>(ceil_div(n, 32), 512), (unsigned)ceil_div(S, 32)),
               dim3(32, 8), 0, st, n, S, x, d, ldd, dmax, xmax, xs, skip);
    return CTQR_OK;
}

ctqr_status refine_keep(int64_t count, const double *xs, double *xbest, const double *hist, hipStream_t st)
{
    if (count <= 0) return CTQR_OK;
    unsigned g = (unsigned)std::min<int64_t>(ceil_div(count, 256), 4096);
    LAUNCH_TRY(refine_keep_kernel, dim3(g), dim3(256), 0, st, count, xs, xbest, hist);
    return CTQR_OK;
}

ctqr_status refine_select(int64_t count, double *x, const double *xbest, const double *hist, ctqr_info *info,
                          hipStream_t st)
{
    if (count <= 0) return CTQR_OK;
    unsigned g = (unsigned)std::min<int64_t>(ceil_div(count, 256), 4096);
    LAUNCH_TRY(refine_select_kernel, dim3(g), dim3(256), 0, st, count, x, xbest, hist, info);
    return CTQR_OK;
}

ctqr_status refine_check(int S, unsigned long long *dmax, unsigned long long *xmax, unsigned long long *smax,
                         double *s0, double tol, int it, int max_iters, int stall_limit, double *hist, int *done,
                         ctqr_info *info, hipStream_t st)
{
    LAUNCH_TRY(refine_check_kernel, dim3(1), dim3(256), 0, st, S, dmax, xmax, smax, s0, tol, it, max_iters,
               stall_limit, hist, done, info);
    return CTQR_OK;
}

ctqr_status slice_absmax(int64_t rows, int S, const double *x, unsigned long long *smax, const int *skip,
                         hipStream_t st)
{
    if (rows <= 0 || S <= 0) return CTQR_OK;
    const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(rows, 4), 1024);
    LAUNCH_TRY(slice_absmax_kernel, dim3(gx, (unsigned)ceil_div(S, 64)), dim3(256), 0, st, rows, S, x, smax, skip);
    return CTQR_OK;
}

template ctqr_status cm_to_rm<double, double>(int64_t, int, const double *, int64_t, double *,
                                              const int *, hipStream_t);
template ctqr_status cm_to_rm<double, float>(int64_t, int, const float *, int64_t, double *,
                                             const int *, hipStream_t);
template ctqr_status rm_to_cm<double, double>(int64_t, int, const double *, double *, int64_t,
                                              const int *, hipStream_t);
template ctqr_status rm_to_cm<float, double>(int64_t, int, const double *, float *, int64_t,
                                             const int *, hipStream_t);
template ctqr_status copy_cm<double, double>(int64_t, int, const double *, int64_t, double *, int64_t,
                                             hipStream_t);
template ctqr_status copy_cm<float, float>(int64_t, int, const float *, int64_t, float *, int64_t, hipStream_t);
template ctqr_status copy_cm<float, double>(int64_t, int, const double *, int64_t, float *, int64_t,
                                            hipStream_t);
template ctqr_status copy_cm<double, float>(int64_t, int, const float *, int64_t, double *, int64_t,
                                            hipStream_t);
template ctqr_status refine_update<float>(int64_t, int, double *, const float *, int64_t,
                                          unsigned long long *, unsigned long long *, double *, const int *,
                                          hipStream_t);
template ctqr_status refine_update<double>(int64_t, int, double *, const double *, int64_t,
                                           unsigned long long *, unsigned long long *, double *, const int *,
                                           hipStream_t);
