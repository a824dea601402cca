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
// One grid barrier per column: after forming reflector j, each workgroup
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

// SL: element type of the slab.  FP64 whenever it fits in LDS; for very tall
// FP32 panels (more rows per workgroup than an FP64 slab can hold) an FP32
// slab, with every sum, norm and reflector scalar still formed in FP64.
// The slab is column-major (column c of the workgroup's rows at
// slab + c * rows_per_wg): the per-column products and updates give one wave
// to a column, its 64 lanes on consecutive rows, and each lane keeps the
// current reflector's values of its rows in registers.
template <typename TS, typename SL>
__global__ __launch_bounds__(PNT)
void panel_qr_kernel(TS *__restrict__ A, int64_t lda, int m, int r0, int w, int rows_per_wg,
                     double *__restrict__ tau_out, double *part, double *part2,
                     double *__restrict__ gram_part, unsigned *bar, ctqr_info *info)
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

    for (int idx = tid; idx < nrows * w; idx += PNT) {
        int c = idx / nrows, rr = idx % nrows;
        slab[c * ldsl + rr] = (SL)A[(int64_t)(r0 + c) * lda + row0 + rr];
    }
    __syncthreads();

    // pivot rows r0 .. r0+w-1 all lie in workgroup 0's slab (rows_per_wg >= 64)
    bool have = false;           // norm and alpha of column j known from the last exchange
    double ss = 0.0, alpha = 0.0;
    bool nonfinite = false;
    for (int j = 0; j < w; ++j) {
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
    __syncthreads();
    {
        const int bi = 16 * (wave / 2), bj = 16 * (wave % 2);
        const int li = lane % 16, kq = lane / 16;
        auto vval = [&](int rr, int c) -> double {
            if (rr >= nrows || c >= w) return 0.0;
            const int g = row0 + rr;
            return g == r0 + c ? 1.0 : (g > r0 + c ? (double)(TS)slab[c * ldsl + rr] : 0.0);
        };
        doublex4 g4 = {0.0, 0.0, 0.0, 0.0};
        for (int k0 = 0; k0 < nrows; k0 += 4) {
            const double a = vval(k0 + kq, bi + li), b = vval(k0 + kq, bj + li);
            g4 = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, g4, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 4; ++r)
            gram_part[(int64_t)wg * PW * PW + (bi + 4 * r + kq) + PW * (bj + li)] = g4[r];
    }
}

// Sum of the per-workgroup Gram partials in a fixed order: 16 entries per
// workgroup, 16 threads per entry each summing every 16th partial, then the
// 16 partial sums in thread order.
__global__ __launch_bounds__(256)
void gram_reduce_kernel(int G, const double *__restrict__ gram_part, double *__restrict__ gram)
{
    __shared__ double red[16][17];
    const int el = threadIdx.x % 16, grp = threadIdx.x / 16;
    const int e = blockIdx.x * 16 + el;
    double s = 0.0;
    for (int q = grp; q < G; q += 16) s += gram_part[(int64_t)q * PW * PW + e];
    red[grp][el] = s;
    __syncthreads();
    if (threadIdx.x < 16) {
        double t = 0.0;
        for (int q = 0; q < 16; ++q) t += red[q][threadIdx.x];
        gram[blockIdx.x * 16 + threadIdx.x] = t;
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
                   TT *__restrict__ Tout, int64_t ldt)
{
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
                     double *part2, double *gram_part, double *gram, unsigned *bar, ctqr_info *info,
                     int ncu, hipStream_t st)
{
    const int mrem = m - r0;
    const int rows = panel_rows_per_wg(mrem, ncu);
    const bool f32slab = sizeof(TS) == 4 && rows > panel_max_rows_per_wg();
    if (rows > (f32slab ? panel_max_rows_per_wg_f32() : panel_max_rows_per_wg())) return CTQR_EUNSUPPORTED;
    const int G = (int)ceil_div(mrem, rows);
    const size_t lds = panel_lds_bytes(rows, f32slab ? sizeof(float) : sizeof(double));
    void *args[] = {&A, (void *)&lda, &m, &r0, &w, (void *)&rows, &tau, &part, &part2, &gram_part, &bar, &info};
    if (f32slab)
        HIP_TRY(hipLaunchCooperativeKernel((const void *)panel_qr_kernel<TS, float>, dim3(G), dim3(PNT), args, lds,
                                           st));
    else
        HIP_TRY(hipLaunchCooperativeKernel((const void *)panel_qr_kernel<TS, double>, dim3(G), dim3(PNT), args,
                                           lds, st));
    LAUNCH_TRY(gram_reduce_kernel, dim3(PW * PW / 16), dim3(256), 0, st, G, (const double *)gram_part, gram);
    return CTQR_OK;
}

ctqr_status panel_setup(int max_rows)
{
    const int l64 = (int)panel_lds_bytes(max_rows, sizeof(double));
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
                   hipStream_t st)
{
    (void)Tw;
    if (nb < 1 || nb > 32 * TB_MAXQ) return CTQR_EINVAL;
    LAUNCH_TRY((tbuild_kernel<TG, TT>), dim3((unsigned)ceil_div(nb, 32)), dim3(256), 0, st, nb, G, ldg, tau, T, ldt);
    return CTQR_OK;
}

template ctqr_status panel_qr<float>(float *, int64_t, int, int, int, double *, double *, double *,
                                     double *, double *, unsigned *, ctqr_info *, int, hipStream_t);
template ctqr_status panel_qr<double>(double *, int64_t, int, int, int, double *, double *, double *,
                                      double *, double *, unsigned *, ctqr_info *, int, hipStream_t);
template ctqr_status tbuild<double, float>(int, const double *, int64_t, const double *, float *, int64_t,
                                           double *, hipStream_t);
template ctqr_status tbuild<double, double>(int, const double *, int64_t, const double *, double *, int64_t,
                                            double *, hipStream_t);
template ctqr_status tbuild<float, float>(int, const float *, int64_t, const double *, float *, int64_t,
                                          double *, hipStream_t);
