// System matrix A on the GPU (Section II-A, Eq. 1; scanner of Table I;
// projection angles of Eq. 2).
//
// a_ij = length of ray i inside pixel j, in pixel pitches.  One thread traces
// one ray with Siddon's parametric method: the ray p0 + alpha (p1 - p0) is
// clipped to the image square, the parameters at which it crosses vertical
// and horizontal grid lines are generated in increasing order by merging the
// two arithmetic sequences, and each interval between consecutive crossings
// is charged to the pixel containing its midpoint (half-open cells, so a ray
// running along a grid line belongs to the cell on its +x/+y side; intervals
// shorter than 1e-12 pitches are dropped).
//
// Outputs, each optional: the dense column-major A (FP64 or FP32, every entry
// written), and the FP64 sparse copy as CSR (entries of a row in traversal
// order) and CSC (rows ascending within a column).  The CSR is built in two
// passes (count, scan, fill); the CSC by counting per column, scanning,
// scattering with atomic slots and sorting each column segment by row, so its
// content does not depend on scheduling.
#include "common.h"
#include "kernels.h"

namespace {

struct Geo {
    int side, n_views, n_bins, sched;
    double R, sdd, half_fan, L;
};

constexpr double ZERO_SEG = 1e-12;
constexpr int SORT_MAX = 4096;    // longest CSC column segment sorted in LDS

__device__ inline double view_angle_deg(const Geo &g, int view)
{
    // Eq. 2: uniform 360/v steps; with the symmetry-breaking schedule, the
    // second, third and fourth quarter turns are offset by +0.5, -0.25 and
    // -0.5 degrees (cumulative jumps +0.5, -0.75, -0.25).
    const int v = g.n_views, i = view + 1;
    double t = (360.0 / v) * (double)(i - 1);
    if (g.sched == 1) {
        if (i > (3 * v) / 4) t += -0.5;
        else if (i > v / 2) t += -0.25;
        else if (i > v / 4) t += 0.5;
    }
    return t;
}

struct Ray {
    double px, py, dx, dy;
};

__device__ inline Ray ray_of(const Geo &g, int i)
{
#pragma clang fp contract(off)
    const int view = i / g.n_bins, bin = i % g.n_bins;
    const double th = view_angle_deg(g, view) * (M_PI / 180.0);
    const double c = cos(th), s = sin(th);
    const double sx = g.R * c, sy = g.R * s;
    const double dcx = sx - g.sdd * c, dcy = sy - g.sdd * s;
    const double pitch = 2.0 * g.sdd * tan(g.half_fan) / g.n_bins;
    const double u = ((double)bin - (g.n_bins - 1) / 2.0) * pitch;
    const double ex = dcx + u * (-s), ey = dcy + u * c;
    Ray r;
    r.px = sx;
    r.py = sy;
    r.dx = ex - sx;
    r.dy = ey - sy;
    return r;
}

// Walk one ray; f(col, length_in_pitches) is called per pixel crossed.
template <typename F>
__device__ inline void siddon_walk(const Geo &g, int ray, F f)
{
#pragma clang fp contract(off)
    const Ray r = ray_of(g, ray);
    const int N = g.side;
    const double delta = g.L / N;
    const double x0 = -g.L / 2.0, y0 = -g.L / 2.0;
    const double xe = x0 + N * delta, ye = y0 + N * delta;
    const double len = sqrt(r.dx * r.dx + r.dy * r.dy);
    double amin = 0.0, amax = 1.0;
    if (r.dx != 0.0) {
        double a0 = (x0 - r.px) / r.dx, a1 = (xe - r.px) / r.dx;
        amin = fmax(amin, fmin(a0, a1));
        amax = fmin(amax, fmax(a0, a1));
    } else if (!(x0 <= r.px && r.px < xe)) {
        return;
    }
    if (r.dy != 0.0) {
        double a0 = (y0 - r.py) / r.dy, a1 = (ye - r.py) / r.dy;
        amin = fmax(amin, fmin(a0, a1));
        amax = fmin(amax, fmax(a0, a1));
    } else if (!(y0 <= r.py && r.py < ye)) {
        return;
    }
    if (!(amax > amin)) return;

    // first grid line beyond amin in the direction of travel, per axis
    const int sx = r.dx > 0.0 ? 1 : -1, sy = r.dy > 0.0 ? 1 : -1;
    int kx = 0, ky = 0;
    if (r.dx != 0.0) {
        double xen = (r.px + amin * r.dx - x0) / delta;
        kx = sx > 0 ? (int)floor(xen) + 1 : (int)ceil(xen) - 1;
        kx = max(-1, min(N + 1, kx));
        while (kx >= 0 && kx <= N && (x0 + kx * delta - r.px) / r.dx <= amin) kx += sx;
        while (kx - sx >= 0 && kx - sx <= N && (x0 + (kx - sx) * delta - r.px) / r.dx > amin) kx -= sx;
    }
    if (r.dy != 0.0) {
        double yen = (r.py + amin * r.dy - y0) / delta;
        ky = sy > 0 ? (int)floor(yen) + 1 : (int)ceil(yen) - 1;
        ky = max(-1, min(N + 1, ky));
        while (ky >= 0 && ky <= N && (y0 + ky * delta - r.py) / r.dy <= amin) ky += sy;
        while (ky - sy >= 0 && ky - sy <= N && (y0 + (ky - sy) * delta - r.py) / r.dy > amin) ky -= sy;
    }
    double acur = amin;
    for (int guard = 0; guard < 4 * N + 8; ++guard) {
        double ax = INFINITY, ay = INFINITY;
        if (r.dx != 0.0 && kx >= 0 && kx <= N) ax = (x0 + kx * delta - r.px) / r.dx;
        if (r.dy != 0.0 && ky >= 0 && ky <= N) ay = (y0 + ky * delta - r.py) / r.dy;
        double anext = fmin(fmin(ax, ay), amax);
        double seg = (anext - acur) * len;
        if (seg > ZERO_SEG * delta) {
            double mid = 0.5 * (acur + anext);
            int ix = (int)floor((r.px + mid * r.dx - x0) / delta);
            int iy = (int)floor((r.py + mid * r.dy - y0) / delta);
            ix = max(0, min(N - 1, ix));
            iy = max(0, min(N - 1, iy));
            f(iy * N + ix, seg / delta);
        }
        if (anext >= amax) break;
        if (ax == anext) kx += sx;
        if (ay == anext) ky += sy;
        acur = anext;
    }
}

__global__ void siddon_count_kernel(Geo g, int m, int64_t *__restrict__ rowcnt)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int64_t c = 0;
    siddon_walk(g, i, [&](int, double) { ++c; });
    rowcnt[i + 1] = c;
    if (i == 0) rowcnt[0] = 0;
}

// Exclusive scan in place of p[1..len] (p[0] = 0 on entry): p becomes the
// prefix sums, p[len] the total.  One workgroup of 1024 threads.
__global__ __launch_bounds__(1024)
void scan_kernel(int64_t len, int64_t *__restrict__ p)
{
    __shared__ int64_t part[1024];
    const int t = threadIdx.x;
    const int64_t chunk = (len + 1023) / 1024;
    const int64_t b = 1 + t * chunk, e = min(len + 1, b + chunk);
    int64_t s = 0;
    for (int64_t i = b; i < e; ++i) s += p[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int64_t v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int64_t run = t > 0 ? part[t - 1] : 0;
    for (int64_t i = b; i < e; ++i) {
        run += p[i];
        p[i] = run;
    }
}

template <typename TA>
__global__ void siddon_fill_kernel(Geo g, int m, const int64_t *__restrict__ rowptr,
                                   int32_t *__restrict__ col, double *__restrict__ val,
                                   int64_t nnz_cap, TA *__restrict__ A, int64_t lda,
                                   int32_t *__restrict__ colcnt, ctqr_info *info)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int64_t pos = rowptr ? rowptr[i] : 0;
    bool over = false;
    siddon_walk(g, i, [&](int j, double a) {
        if (A) A[(int64_t)j * lda + i] = (TA)a;
        if (rowptr) {
            if (pos < nnz_cap) {
                col[pos] = j;
                val[pos] = a;
                if (colcnt) atomicAdd(&colcnt[j], 1);
            } else {
                over = true;
            }
            ++pos;
        }
    });
    if (over) info_event(info, CTQR_CAPACITY, -1);
}

__global__ void nnz_kernel(int m, const int64_t *__restrict__ rowptr, ctqr_info *info)
{
    info->nnz = rowptr[m];
}

__global__ void colcnt_to_ptr_kernel(int n, const int32_t *__restrict__ cnt, int64_t *__restrict__ colptr)
{
    int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) colptr[j + 1] = cnt[j];
    if (j == 0) colptr[0] = 0;
}

__global__ void csc_scatter_kernel(int m, const int64_t *__restrict__ rowptr,
                                   const int32_t *__restrict__ col, const double *__restrict__ val,
                                   int64_t nnz_cap, const int64_t *__restrict__ colptr,
                                   int32_t *__restrict__ fill, int32_t *__restrict__ row,
                                   double *__restrict__ cval)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= m) return;
    int64_t e = min(rowptr[i + 1], nnz_cap);
    for (int64_t k = rowptr[i]; k < e; ++k) {
        int j = col[k];
        int64_t p = colptr[j] + atomicAdd(&fill[j], 1);
        if (p < nnz_cap) {
            row[p] = i;
            cval[p] = val[k];
        }
    }
}

// Sort one column segment of the CSC by row (bitonic, in LDS).
__global__ __launch_bounds__(256)
void csc_sort_kernel(int n, const int64_t *__restrict__ colptr, int64_t nnz_cap,
                     int32_t *__restrict__ row, double *__restrict__ cval, ctqr_info *info)
{
    __shared__ int32_t kr[SORT_MAX];
    __shared__ double kv[SORT_MAX];
    const int j = blockIdx.x;
    const int64_t b = colptr[j], e = min(colptr[j + 1], nnz_cap);
    const int len = (int)max((int64_t)0, e - b);
    if (len > SORT_MAX) {
        if (threadIdx.x == 0) info_event(info, CTQR_CAPACITY, j);
        return;
    }
    int p2 = 1;
    while (p2 < len) p2 <<= 1;
    for (int t = threadIdx.x; t < p2; t += 256) {
        kr[t] = t < len ? row[b + t] : INT32_MAX;
        kv[t] = t < len ? cval[b + t] : 0.0;
    }
    __syncthreads();
    for (int k = 2; k <= p2; k <<= 1)
        for (int s = k >> 1; s > 0; s >>= 1) {
            for (int t = threadIdx.x; t < p2; t += 256) {
                int o = t ^ s;
                if (o > t) {
                    bool up = (t & k) == 0;
                    if ((kr[t] > kr[o]) == up) {
                        int32_t r = kr[t]; kr[t] = kr[o]; kr[o] = r;
                        double v = kv[t]; kv[t] = kv[o]; kv[o] = v;
                    }
                }
            }
            __syncthreads();
        }
    for (int t = threadIdx.x; t < len; t += 256) {
        row[b + t] = kr[t];
        cval[b + t] = kv[t];
    }
}

template <typename TA>
__global__ void zero_dense_kernel(TA *__restrict__ A, int64_t lda, int64_t m, int64_t n)
{
    int64_t total = lda * n;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
         e += (int64_t)gridDim.x * blockDim.x)
        A[e] = TA(0);
    (void)m;
}

__global__ void zero_i32_kernel(int32_t *__restrict__ p, int64_t n)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n;
         e += (int64_t)gridDim.x * blockDim.x)
        p[e] = 0;
}

// Columns [c0, c1) of the dense A from the CSC copy: column c0 + q of A goes
// to out + q ldo (zeros elsewhere).  One wave per column.
template <typename TA>
__global__ __launch_bounds__(256)
void csc_to_dense_kernel(int c0, int c1, const int64_t *__restrict__ colptr, const int32_t *__restrict__ row,
                         const double *__restrict__ cval, TA *__restrict__ out, int64_t ldo)
{
    const int j = c0 + (int)blockIdx.x * 4 + (int)threadIdx.x / 64;
    if (j >= c1) return;
    TA *o = out + (int64_t)(j - c0) * ldo;
    for (int64_t k = colptr[j] + threadIdx.x % 64; k < colptr[j + 1]; k += 64) o[row[k]] = (TA)cval[k];
}

// Joseph's projector (sinogram simulation): the ray is sampled once per
// pixel column when it runs closer to the x axis (else once per pixel row),
// at the line through the pixel centres; the image there is linearly
// interpolated between the two nearest pixel centres of that column (row),
// pixels outside the image counting as zero, and each sample is weighted by
// the ray length between consecutive column (row) lines, in pixel pitches.
// Thread per (ray, slice); X column-major n x S (pixel iy * side + ix).
__global__ __launch_bounds__(256)
void joseph_kernel(Geo g, int m, const double *__restrict__ X, int64_t ldx, double *__restrict__ B, int64_t ldb)
{
#pragma clang fp contract(off)
    const int i = (int)blockIdx.x * 256 + (int)threadIdx.x;
    const int s = blockIdx.y;
    if (i >= m) return;
    const Ray r = ray_of(g, i);
    const int N = g.side;
    const double delta = g.L / N;
    const double x0 = -g.L / 2.0, y0 = -g.L / 2.0;
    const double *img = X + (int64_t)s * ldx;
    const double len = sqrt(r.dx * r.dx + r.dy * r.dy);
    double total = 0.0;
    if (fabs(r.dx) >= fabs(r.dy)) {
        const double w = len / fabs(r.dx);
        for (int ix = 0; ix < N; ++ix) {
            const double t = (x0 + (ix + 0.5) * delta - r.px) / r.dx;
            const double v = (r.py + t * r.dy - y0) / delta - 0.5;
            const double fl = floor(v);
            const double f = v - fl;
            const int iy = (int)fl;
            const double a = (iy >= 0 && iy < N) ? img[(int64_t)iy * N + ix] : 0.0;
            const double b = (iy + 1 >= 0 && iy + 1 < N) ? img[(int64_t)(iy + 1) * N + ix] : 0.0;
            total += w * ((1.0 - f) * a + f * b);
        }
    } else {
        const double w = len / fabs(r.dy);
        for (int iy = 0; iy < N; ++iy) {
            const double t = (y0 + (iy + 0.5) * delta - r.py) / r.dy;
            const double u = (r.px + t * r.dx - x0) / delta - 0.5;
            const double fl = floor(u);
            const double f = u - fl;
            const int ix = (int)fl;
            const double a = (ix >= 0 && ix < N) ? img[(int64_t)iy * N + ix] : 0.0;
            const double b = (ix + 1 >= 0 && ix + 1 < N) ? img[(int64_t)iy * N + ix + 1] : 0.0;
            total += w * ((1.0 - f) * a + f * b);
        }
    }
    B[(int64_t)s * ldb + i] = total;
}

}  // namespace

size_t siddon_workspace(const ctqr_geometry *g)
{
    int64_t n = (int64_t)g->side * g->side;
    return (size_t)(2 * n + 64) * sizeof(int32_t);
}

ctqr_status joseph_project(const ctqr_geometry *gp, int S, const double *X, int64_t ldx, double *B, int64_t ldb,
                           hipStream_t st)
{
    Geo g;
    g.side = gp->side;
    g.n_views = gp->n_views;
    g.n_bins = gp->n_bins;
    g.sched = gp->angle_schedule;
    g.R = gp->src_iso_cm;
    g.sdd = gp->src_det_cm;
    g.half_fan = gp->fan_deg * (M_PI / 180.0) / 2.0;
    g.L = gp->fov_side_cm;
    const int m = g.n_views * g.n_bins;
    LAUNCH_TRY(joseph_kernel, dim3((unsigned)ceil_div(m, 256), (unsigned)S), dim3(256), 0, st, g, m, X, ldx, B, ldb);
    return CTQR_OK;
}

ctqr_status siddon_build(const ctqr_geometry *gp, int dtype, void *A, int64_t lda, ctqr_sparse *sp,
                         void *work, size_t work_bytes, ctqr_info *info, hipStream_t st)
{
    Geo g;
    g.side = gp->side;
    g.n_views = gp->n_views;
    g.n_bins = gp->n_bins;
    g.sched = gp->angle_schedule;
    g.R = gp->src_iso_cm;
    g.sdd = gp->src_det_cm;
    g.half_fan = gp->fan_deg * (M_PI / 180.0) / 2.0;
    g.L = gp->fov_side_cm;
    const int m = g.n_views * g.n_bins;
    const int64_t n = (int64_t)g.side * g.side;
    if (work_bytes < siddon_workspace(gp)) return CTQR_ENOMEM;
    int32_t *colcnt = (int32_t *)work;
    int32_t *colfill = colcnt + n;
    const dim3 rb(256), rg((unsigned)ceil_div(m, 256));

    if (A) {
        unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(lda * n, 256), 1 << 20);
        if (dtype == CTQR_F64)
            LAUNCH_TRY(zero_dense_kernel<double>, dim3(blocks), dim3(256), 0, st, (double *)A, lda, (int64_t)m, n);
        else
            LAUNCH_TRY(zero_dense_kernel<float>, dim3(blocks), dim3(256), 0, st, (float *)A, lda, (int64_t)m, n);
    }
    int64_t *rowptr = sp ? sp->rowptr : nullptr;
    if (sp) {
        LAUNCH_TRY(siddon_count_kernel, rg, rb, 0, st, g, m, rowptr);
        LAUNCH_TRY(scan_kernel, dim3(1), dim3(1024), 0, st, (int64_t)m, rowptr);
        LAUNCH_TRY(nnz_kernel, dim3(1), dim3(1), 0, st, m, (const int64_t *)rowptr, info);
        LAUNCH_TRY(zero_i32_kernel, dim3((unsigned)ceil_div(2 * n, 256)), dim3(256), 0, st, colcnt, 2 * n);
    }
    int32_t *cc = sp ? colcnt : nullptr;
    int32_t *colp = sp ? sp->col : nullptr;
    double *valp = sp ? sp->val : nullptr;
    int64_t cap = sp ? sp->nnz_cap : 0;
    if (dtype == CTQR_F64)
        LAUNCH_TRY(siddon_fill_kernel<double>, rg, rb, 0, st, g, m, (const int64_t *)rowptr, colp, valp,
                   cap, (double *)A, lda, cc, info);
    else
        LAUNCH_TRY(siddon_fill_kernel<float>, rg, rb, 0, st, g, m, (const int64_t *)rowptr, colp, valp,
                   cap, (float *)A, lda, cc, info);
    if (sp && sp->colptr) {
        LAUNCH_TRY(colcnt_to_ptr_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, st, (int)n,
                   (const int32_t *)colcnt, sp->colptr);
        LAUNCH_TRY(scan_kernel, dim3(1), dim3(1024), 0, st, n, sp->colptr);
        LAUNCH_TRY(csc_scatter_kernel, rg, rb, 0, st, m, (const int64_t *)rowptr, (const int32_t *)sp->col,
                   (const double *)sp->val, cap, (const int64_t *)sp->colptr, colfill, sp->row, sp->cval);
        LAUNCH_TRY(csc_sort_kernel, dim3((unsigned)n), dim3(256), 0, st, (int)n,
                   (const int64_t *)sp->colptr, cap, sp->row, sp->cval, info);
    }
    return CTQR_OK;
}

ctqr_status sparse_to_dense_cols(const ctqr_sparse *sp, int dtype, int c0, int c1, void *A, int64_t lda,
                                 hipStream_t st)
{
    const int64_t cols = c1 - c0;
    if (cols <= 0) return CTQR_OK;
    unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(lda * cols, 256), 1 << 20);
    const dim3 g((unsigned)ceil_div(cols, 4)), b(256);
    if (dtype == CTQR_F64) {
        LAUNCH_TRY(zero_dense_kernel<double>, dim3(blocks), dim3(256), 0, st, (double *)A, lda, lda, cols);
        LAUNCH_TRY(csc_to_dense_kernel<double>, g, b, 0, st, c0, c1, (const int64_t *)sp->colptr,
                   (const int32_t *)sp->row, (const double *)sp->cval, (double *)A, lda);
    } else {
        LAUNCH_TRY(zero_dense_kernel<float>, dim3(blocks), dim3(256), 0, st, (float *)A, lda, lda, cols);
        LAUNCH_TRY(csc_to_dense_kernel<float>, g, b, 0, st, c0, c1, (const int64_t *)sp->colptr,
                   (const int32_t *)sp->row, (const double *)sp->cval, (float *)A, lda);
    }
    return CTQR_OK;
}
