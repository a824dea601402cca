// Preconditioned conjugate gradients on the normal equations, the Krylov
// form of the corrected semi-normal-equations refinement: the same FP64
// residuals r = B - A x and s = A^T r against the sparse A, the same
// preconditioner (R^T R)^-1 applied by the two triangular solves with the
// factor's R, but the corrections are combined as conjugate directions
// instead of added one by one.  Every slice runs its own iteration, so all
// scalars are per slice.  Vectors are row-major (row i holds the S slices).
//
// Per iteration (the triangular solves and the sparse products are launched
// by the driver):
//   z = (R^T R)^-1 s,  gamma = s.z,
//   beta = max(0, (gamma - s.z_prev) / gamma_prev)     (Polak-Ribiere; 0 first)
//   p = z + beta p,  q = A p,  alpha = gamma / q.q,  x += alpha p.
// The Polak-Ribiere coefficient keeps the directions useful when the
// preconditioner is applied in FP32 and so changes slightly between calls.
#include "common.h"
#include "kernels.h"

namespace {

constexpr int DOT_THREADS = 256;

// partial[b][s] = sum over the rows of block b (rows b R .. (b+1) R - 1) of
// x[i, s] y[i, s]; threads cover (slice, row offset) pairs and combine the
// row offsets in a fixed order.
__global__ __launch_bounds__(DOT_THREADS)
void slice_dot_partial_kernel(int64_t rows, int S, int64_t rows_per_block, const double *__restrict__ x,
                              const double *__restrict__ y, double *__restrict__ partial, const int *skip)
{
    if (skip && *skip) return;
    __shared__ double red[DOT_THREADS];
    const int64_t r0 = (int64_t)blockIdx.x * rows_per_block;
    const int64_t r1 = min(rows, r0 + rows_per_block);
    for (int s0 = 0; s0 < S; s0 += DOT_THREADS) {
        const int sw = min(DOT_THREADS, S - s0);     // slices in this chunk
        const int rt = DOT_THREADS / sw;             // row offsets in parallel
        const int s = s0 + (int)threadIdx.x % sw, ro = (int)threadIdx.x / sw;
        double acc = 0.0;
        if (ro < rt)
            for (int64_t i = r0 + ro; i < r1; i += rt) acc += x[i * S + s] * y[i * S + s];
        red[threadIdx.x] = ro < rt ? acc : 0.0;
        __syncthreads();
        if (ro == 0) {
            double v = red[threadIdx.x];
            for (int k = 1; k < rt; ++k) v += red[threadIdx.x + k * sw];
            partial[(int64_t)blockIdx.x * S + s] = v;
        }
        __syncthreads();
    }
}

// out[s] = sum_b partial[b][s] in block order
__global__ void slice_dot_final_kernel(int S, int nblocks, const double *__restrict__ partial,
                                       double *__restrict__ out, const int *skip)
{
    if (skip && *skip) return;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    double v = 0.0;
    for (int b = 0; b < nblocks; ++b) v += partial[(int64_t)b * S + s];
    out[s] = v;
}

// gamma = s.z, beta from Polak-Ribiere (0 on the first iteration)
__global__ void pcg_beta_kernel(int S, int first, const double *__restrict__ sz, const double *__restrict__ szp,
                                double *__restrict__ gamma, double *__restrict__ beta, const int *skip)
{
    if (skip && *skip) return;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    const double g = sz[s];
    double b = 0.0;
    if (!first && gamma[s] > 0.0) b = fmax(0.0, (g - szp[s]) / gamma[s]);
    beta[s] = b;
    gamma[s] = g;
}

// alpha = gamma / q.q (0 for a slice with no direction left)
__global__ void pcg_alpha_kernel(int S, const double *__restrict__ gamma, const double *__restrict__ qq,
                                 double *__restrict__ alpha, const int *skip)
{
    if (skip && *skip) return;
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s >= S) return;
    alpha[s] = qq[s] > 0.0 ? gamma[s] / qq[s] : 0.0;
}

// p = z + beta p
__global__ void pcg_direction_kernel(int64_t total, int S, const double *__restrict__ z,
                                     const double *__restrict__ beta, double *__restrict__ p, const int *skip)
{
    if (skip && *skip) return;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = z[e] + beta[e % S] * p[e];
}

__device__ inline unsigned long long abs_bits(double v)
{
    // |v| as an unsigned key ordered like |v| (non-negative doubles order as
    // their bit patterns); NaN maps above every finite value
    const double a = fabs(v);
    return a == a ? (unsigned long long)__double_as_longlong(a) : ~0ull;
}

// x += alpha p; per-slice max |alpha p| and max |x| (bit patterns, atomic max
// after a block reduction)
__global__ __launch_bounds__(256)
void pcg_step_kernel(int64_t rows, int S, double *__restrict__ x, const double *__restrict__ p,
                     const double *__restrict__ alpha, unsigned long long *dmax, unsigned long long *xmax,
                     double *__restrict__ xs, const int *skip)
{
    if (skip && *skip) return;
    __shared__ unsigned long long md[256], mx[256];
    for (int s0 = 0; s0 < S; s0 += 256) {
        const int sw = min(256, S - s0), rt = 256 / sw;
        const int s = s0 + (int)threadIdx.x % sw, ro = (int)threadIdx.x / sw;
        unsigned long long dm = 0, xm = 0;
        if (ro < rt) {
            const double a = alpha[s];
            for (int64_t i = (int64_t)blockIdx.x * rt + ro; i < rows; i += (int64_t)gridDim.x * rt) {
                const double d = a * p[i * S + s];
                const double xo = x[i * S + s];
                if (xs) xs[i * S + s] = xo;
                const double xv = xo + d;
                x[i * S + s] = xv;
                const unsigned long long bd = abs_bits(d), bx = abs_bits(xv);
                dm = bd > dm ? bd : dm;
                xm = bx > xm ? bx : xm;
            }
        }
        md[threadIdx.x] = dm;
        mx[threadIdx.x] = xm;
        __syncthreads();
        if (ro == 0) {
            for (int k = 1; k < rt; ++k) {
                dm = md[threadIdx.x + k * sw] > dm ? md[threadIdx.x + k * sw] : dm;
                xm = mx[threadIdx.x + k * sw] > xm ? mx[threadIdx.x + k * sw] : xm;
            }
            atomicMax(&dmax[s], dm);
            atomicMax(&xmax[s], xm);
        }
        __syncthreads();
    }
}

}  // namespace

size_t slice_dot_partial_elems(int S) { return (size_t)PCG_DOT_BLOCKS * S; }

ctqr_status slice_dot(int64_t rows, int S, const double *x, const double *y, double *partial, double *out,
                      const int *skip, hipStream_t st)
{
    const int64_t rpb = ceil_div(rows, PCG_DOT_BLOCKS);
    LAUNCH_TRY(slice_dot_partial_kernel, dim3(PCG_DOT_BLOCKS), dim3(DOT_THREADS), 0, st, rows, S, rpb, x, y,
               partial, skip);
    LAUNCH_TRY(slice_dot_final_kernel, dim3((unsigned)ceil_div(S, 256)), dim3(256), 0, st, S, PCG_DOT_BLOCKS,
               (const double *)partial, out, skip);
    return CTQR_OK;
}

ctqr_status pcg_beta(int S, int first, const double *sz, const double *szp, double *gamma, double *beta,
                     const int *skip, hipStream_t st)
{
    LAUNCH_TRY(pcg_beta_kernel, dim3((unsigned)ceil_div(S, 256)), dim3(256), 0, st, S, first, sz, szp, gamma, beta,
               skip);
    return CTQR_OK;
}

ctqr_status pcg_alpha(int S, const double *gamma, const double *qq, double *alpha, const int *skip, hipStream_t st)
{
    LAUNCH_TRY(pcg_alpha_kernel, dim3((unsigned)ceil_div(S, 256)), dim3(256), 0, st, S, gamma, qq, alpha, skip);
    return CTQR_OK;
}

ctqr_status pcg_direction(int64_t rows, int S, const double *z, const double *beta, double *p, const int *skip,
                          hipStream_t st)
{
    const int64_t total = rows * S;
    LAUNCH_TRY(pcg_direction_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(total, 256), 4096)), dim3(256), 0,
               st, total, S, z, beta, p, skip);
    return CTQR_OK;
}

ctqr_status pcg_step(int64_t rows, int S, double *x, const double *p, const double *alpha, unsigned long long *dmax,
                     unsigned long long *xmax, double *xs, const int *skip, hipStream_t st)
{
    const int rt = 256 / std::min(256, S);
    const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(rows, rt), 512);
    LAUNCH_TRY(pcg_step_kernel, dim3(blocks), dim3(256), 0, st, rows, S, x, p, alpha, dmax, xmax, xs, skip);
    return CTQR_OK;
}
