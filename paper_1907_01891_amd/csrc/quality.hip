// Image-quality metrics of the reconstructions (Section II-B): PSNR (Eq. 5
// and Eq. 6) and the mean SSIM (Eq. 7) of each slice against its reference
// image.  One workgroup per slice, every sum in a fixed order and tree, so the
// results do not depend on scheduling.
//
// SSIM windows: every 11 x 11 window inside the side x side image, weighted by
// the Gaussian of standard deviation 1.5 pixels (normalised to sum 1) for the
// means, variances and covariance; c1 = (0.01 L)^2, c2 = (0.03 L)^2 with L the
// data range (the caller's, or max - min of the reference image).
#include "common.h"
#include "kernels.h"

namespace {

constexpr int QT = 256;
constexpr int WIN = 11;

__device__ inline double block_sum(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int k = QT / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    const double out = red[0];
    __syncthreads();
    return out;
}

__device__ inline double block_max(double v, double *red)
{
    red[threadIdx.x] = v;
    __syncthreads();
    for (int k = QT / 2; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] = fmax(red[threadIdx.x], red[threadIdx.x + k]);
        __syncthreads();
    }
    const double out = red[0];
    __syncthreads();
    return out;
}

__global__ __launch_bounds__(QT)
void image_quality_kernel(int side, const double *__restrict__ Xref, int64_t ldr, const double *__restrict__ X,
                          int64_t ldx, double data_range, int S, double *__restrict__ out)
{
    __shared__ double red[QT];
    __shared__ double wg[WIN];
    const int s = blockIdx.x;
    const double *ref = Xref + (int64_t)s * ldr;
    const double *img = X + (int64_t)s * ldx;
    const int64_t n = (int64_t)side * side;
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int k = 0; k < WIN; ++k) {
            const double r = k - (WIN - 1) / 2.0;
            wg[k] = exp(-r * r / (2.0 * 1.5 * 1.5));
            sum += wg[k];
        }
        for (int k = 0; k < WIN; ++k) wg[k] /= sum;   // the 2-D weights are wg[a] wg[b], sum 1
    }
    // PSNR: MSE over the image, MAX = largest reference value
    double se = 0.0, mx = -INFINITY, mn = INFINITY;
    for (int64_t p = threadIdx.x; p < n; p += QT) {
        const double a = ref[p], d = a - img[p];
        se += d * d;
        mx = fmax(mx, a);
        mn = fmin(mn, a);
    }
    const double sse = block_sum(se, red);
    const double rmax = block_max(mx, red);
    const double rmin = -block_max(-mn, red);
    const double mse = sse / (double)n;
    const double L = data_range > 0.0 ? data_range : rmax - rmin;
    const double c1 = (0.01 * L) * (0.01 * L), c2 = (0.03 * L) * (0.03 * L);
    // SSIM over the windows
    const int nw = side - WIN + 1;
    double acc = 0.0;
    for (int64_t w = threadIdx.x; nw > 0 && w < (int64_t)nw * nw; w += QT) {
        const int p0 = (int)(w / nw), q0 = (int)(w % nw);   // window rows p0.., columns q0..
        double mxw = 0.0, myw = 0.0, sxx = 0.0, syy = 0.0, sxy = 0.0;
        for (int a = 0; a < WIN; ++a) {
            const double *ra = ref + (int64_t)(p0 + a) * side + q0;
            const double *ia = img + (int64_t)(p0 + a) * side + q0;
            for (int b = 0; b < WIN; ++b) {
                const double wt = wg[a] * wg[b];
                const double x = ra[b], y = ia[b];
                mxw += wt * x;
                myw += wt * y;
                sxx += wt * x * x;
                syy += wt * y * y;
                sxy += wt * x * y;
            }
        }
        const double vx = sxx - mxw * mxw, vy = syy - myw * myw, cxy = sxy - mxw * myw;
        acc += (2.0 * mxw * myw + c1) * (2.0 * cxy + c2) / ((mxw * mxw + myw * myw + c1) * (vx + vy + c2));
    }
    const double ssum = block_sum(acc, red);
    if (threadIdx.x == 0) {
        out[s] = mse > 0.0 ? 10.0 * log10(rmax * rmax / mse) : INFINITY;
        out[S + s] = nw > 0 ? ssum / ((double)nw * nw) : NAN;
    }
}

}  // namespace

ctqr_status image_quality(int side, int S, const double *Xref, int64_t ldr, const double *X, int64_t ldx,
                          double data_range, double *out, hipStream_t st)
{
    LAUNCH_TRY(image_quality_kernel, dim3((unsigned)S), dim3(QT), 0, st, side, Xref, ldr, X, ldx, data_range, S, out);
    return CTQR_OK;
}
