// Kernels of the condition-number estimate: start vectors, per-column dot
// products and scaling, and the running maxima of the Rayleigh quotients.
// Vectors are column-major (rows x S, leading dimension ld) unless a kernel
// says row-major (rows x S, slice index fastest).
#include "common.h"
#include "kernels.h"

namespace {

// splitmix64 finaliser: a counter-based hash, so every start vector is a
// fixed function of (row, column) and the estimate is reproducible.
__device__ inline uint64_t mix64(uint64_t z)
{
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

// x[r, s] uniform in [-1, 1): column-major (leading dimension ldx) or, with
// RM, row-major
template <typename T, bool RM>
__global__ void cond_start_kernel(int64_t rows, int S, T *__restrict__ x, int64_t ldx, uint64_t seed)
{
    const int64_t total = rows * S;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int64_t r = RM ? e / S : e % rows;
        const int s = (int)(RM ? e % S : e / rows);
        const uint64_t h = mix64(seed ^ mix64(((uint64_t)s << 40) ^ (uint64_t)r));
        const T v = (T)((double)(h >> 11) * (1.0 / 4503599627370496.0) - 1.0);
        if (RM)
            x[e] = v;
        else
            x[(int64_t)s * ldx + r] = v;
    }
}

// out[s] = sum_r x[r, s] y[r, s] in FP64: one workgroup per column, a fixed
// strided order and tree, so the result does not depend on timing.
template <typename TX, typename TY>
__global__ __launch_bounds__(256)
void col_dot_kernel(int64_t rows, const TX *__restrict__ x, int64_t ldx, const TY *__restrict__ y, int64_t ldy,
                    double *__restrict__ out)
{
    __shared__ double red[256];
    const int s = blockIdx.x;
    const TX *xs = x + (int64_t)s * ldx;
    const TY *ys = y + (int64_t)s * ldy;
    double acc = 0.0;
    for (int64_t r = threadIdx.x; r < rows; r += 256) acc += (double)xs[r] * (double)ys[r];
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if (threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[s] = red[0];
}

// dst[:, s] = src[:, s] / sqrt(dots[s]) (columns of norm zero are left zero)
template <typename TD, typename TS>
__global__ void col_scale_kernel(int64_t rows, const TS *__restrict__ src, int64_t lds, const double *__restrict__ dots,
                                 TD *__restrict__ dst, int64_t ldd)
{
    const int s = blockIdx.y;
    const double d = dots[s];
    const double f = d > 0.0 ? 1.0 / sqrt(d) : 0.0;
    for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows;
         r += (int64_t)gridDim.x * blockDim.x)
        dst[(int64_t)s * ldd + r] = (TD)((double)src[(int64_t)s * lds + r] * f);
}

// x[r, s] *= 1 / sqrt(dots[s]) for a row-major rows x S array
__global__ void rm_scale_kernel(int64_t rows, int S, double *__restrict__ x, const double *__restrict__ dots)
{
    const int64_t total = rows * S;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x) {
        const double d = dots[e % S];
        x[e] = d > 0.0 ? x[e] / sqrt(d) : 0.0;
    }
}

// est[slot] = max(est[slot], max_s q[s]) (NaN is kept: it marks a failure)
__global__ void cond_max_kernel(int S, const double *__restrict__ q, double *est, int slot)
{
    if (threadIdx.x != 0) return;
    double m = est[slot];
    for (int s = 0; s < S; ++s) {
        const double v = q[s];
        if (v != v) m = v;
        else if (m == m && v > m) m = v;
    }
    est[slot] = m;
}

// out = [sigma_max, sigma_min, kappa] from the largest Rayleigh quotients of
// A^T A (est[0]) and of (R^T R)^-1 (est[1]).
__global__ void cond_finish_kernel(const double *est, double *out)
{
    if (threadIdx.x != 0) return;
    const double smax = sqrt(est[0]);
    const double smin = est[1] > 0.0 ? 1.0 / sqrt(est[1]) : 0.0;
    out[0] = smax;
    out[1] = smin;
    out[2] = smin > 0.0 ? smax / smin : INFINITY;
}

unsigned grid_rows(int64_t rows) { return (unsigned)std::min<int64_t>(ceil_div(rows, 256), 1024); }

}  // namespace

template <typename T>
ctqr_status cond_start(int64_t rows, int S, T *x, int64_t ldx, uint64_t seed, hipStream_t st)
{
    const unsigned g = (unsigned)std::min<int64_t>(ceil_div(rows * S, 256), 4096);
    if (ldx == 0)
        LAUNCH_TRY((cond_start_kernel<T, true>), dim3(g), dim3(256), 0, st, rows, S, x, ldx, seed);
    else
        LAUNCH_TRY((cond_start_kernel<T, false>), dim3(g), dim3(256), 0, st, rows, S, x, ldx, seed);
    return CTQR_OK;
}

template <typename TX, typename TY>
ctqr_status col_dot(int64_t rows, int S, const TX *x, int64_t ldx, const TY *y, int64_t ldy, double *out,
                    hipStream_t st)
{
    LAUNCH_TRY((col_dot_kernel<TX, TY>), dim3((unsigned)S), dim3(256), 0, st, rows, x, ldx, y, ldy, out);
    return CTQR_OK;
}

template <typename TD, typename TS>
ctqr_status col_scale(int64_t rows, int S, const TS *src, int64_t lds, const double *dots, TD *dst, int64_t ldd,
                      hipStream_t st)
{
    LAUNCH_TRY((col_scale_kernel<TD, TS>), dim3(grid_rows(rows), (unsigned)S), dim3(256), 0, st, rows, src, lds,
               dots, dst, ldd);
    return CTQR_OK;
}

ctqr_status rm_scale(int64_t rows, int S, double *x, const double *dots, hipStream_t st)
{
    const unsigned g = (unsigned)std::min<int64_t>(ceil_div(rows * S, 256), 4096);
    LAUNCH_TRY(rm_scale_kernel, dim3(g), dim3(256), 0, st, rows, S, x, dots);
    return CTQR_OK;
}

ctqr_status cond_max(int S, const double *q, double *est, int slot, hipStream_t st)
{
    LAUNCH_TRY(cond_max_kernel, dim3(1), dim3(64), 0, st, S, q, est, slot);
    return CTQR_OK;
}

ctqr_status cond_finish(const double *est, double *out, hipStream_t st)
{
    LAUNCH_TRY(cond_finish_kernel, dim3(1), dim3(64), 0, st, est, out);
    return CTQR_OK;
}

template ctqr_status cond_start<double>(int64_t, int, double *, int64_t, uint64_t, hipStream_t);
template ctqr_status cond_start<float>(int64_t, int, float *, int64_t, uint64_t, hipStream_t);
template ctqr_status col_dot<double, double>(int64_t, int, const double *, int64_t, const double *, int64_t,
                                             double *, hipStream_t);
template ctqr_status col_dot<float, float>(int64_t, int, const float *, int64_t, const float *, int64_t, double *,
                                           hipStream_t);
template ctqr_status col_scale<double, double>(int64_t, int, const double *, int64_t, const double *, double *,
                                               int64_t, hipStream_t);
template ctqr_status col_scale<float, float>(int64_t, int, const float *, int64_t, const double *, float *, int64_t,
                                             hipStream_t);
