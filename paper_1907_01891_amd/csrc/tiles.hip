// Algorithm-by-blocks QR factorization and solve (Section II-C): the matrix
// is cut into b x b blocks (b <= 64; the last block row and column may be
// smaller) and processed by four task types, each working on a few blocks,
// plus the solve's block substitution and block product:
//   dense_qr(k)          Compute_dense_QR: Householder QR of A_kk, its
//                        compact-WY factor S_kk (H_1 ... H_c = I - V S V^T).
//   td_qr(i, k)          Compute_TD_QR: QR of the triangle R_kk stacked on the
//                        dense A_ik; reflectors [e_p; v_p], v_p into A_ik, R_kk
//                        updated, S_ik for U = [I; A_ik].
//   apply_dense(k, C)    Apply_left_Qt_of_dense_QR: C <- (I - V S V^T)^T C.
//   apply_td(i, k, F, G) Apply_left_Qt_of_TD_QR: [F; G] <- (I - U S U^T)^T [F; G].
//   trsm(i)              X_i = R_ii^-1 B_i (Trsm_lunn).
//   gemm(i, j)           B_i -= R_ij X_j (Gemm_nn_mo).
// One workgroup runs one task (or one task on a chunk of right-hand-side
// columns) with its blocks in LDS, FP64 throughout.  The host orders the
// tasks as the paper's task tables do, groups them into dependency levels and
// launches each level's tasks of one type together.
//
// Householder vectors follow the larfg convention (beta = -sign(alpha) norm,
// sign(0) = +1, tau = (beta - alpha) / beta, v = x / (alpha - beta), tau = 0
// for x = 0) and S is built by the larft recurrence
// S_pp = tau_p, S_{0:p, p} = -tau_p S_{0:p, 0:p} (U^T u_p)_{0:p}.
#include <algorithm>
#include <unordered_map>
#include <vector>

#include "common.h"
#include "kernels.h"

namespace {

constexpr int TB = 64;          // largest block size
constexpr int LD = TB + 1;      // LDS leading dimension (column-major tiles)
constexpr int NT = 256;         // threads per workgroup
constexpr int RHS_CHUNK = 64;   // right-hand-side columns per solve workgroup

struct Dims {
    int m, n, b, mt, nt;
    __device__ int rows(int i) const { return min(b, m - i * b); }
    __device__ int cols(int j) const { return min(b, n - j * b); }
};

__device__ inline double *tile_ptr(double *A, int64_t lda, const Dims &d, int i, int j)
{
    return A + (int64_t)(j * d.b) * lda + (int64_t)i * d.b;
}

// S factor of block (i, k), i >= k: b x b column-major at Sf + ((k * mt) + i) b^2
__device__ inline double *s_ptr(double *Sf, const Dims &d, int i, int k)
{
    return Sf + ((int64_t)k * d.mt + i) * d.b * d.b;
}

__device__ inline void load_tile(double *L, const double *g, int64_t ld, int r, int c)
{
    for (int e = threadIdx.x; e < TB * TB; e += NT) {
        const int q = e / TB, i = e % TB;
        L[q * LD + i] = (i < r && q < c) ? g[(int64_t)q * ld + i] : 0.0;
    }
}

__device__ inline void store_tile(const double *L, double *g, int64_t ld, int r, int c)
{
    for (int e = threadIdx.x; e < TB * TB; e += NT) {
        const int q = e / TB, i = e % TB;
        if (i < r && q < c) g[(int64_t)q * ld + i] = L[q * LD + i];
    }
}

// Sum over the 64 lanes of a wave (butterfly: every lane gets the total).
__device__ inline double wave_sum(double v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

// larfg on (alpha, x[0..len)): beta, tau, and x scaled in place to v.
// Runs in wave 0; x in LDS with stride 1.
__device__ inline void larfg_wave0(double *alpha_p, double *x, int len, double *tau_out)
{
    const int lane = threadIdx.x;
    double s = 0.0;
    for (int i = lane; i < len; i += CTQR_WAVE) s += x[i] * x[i];
    s = wave_sum(s);
    const double alpha = *alpha_p;
    double beta = alpha, tau = 0.0;
    if (s != 0.0) {
        beta = -copysign(sqrt(alpha * alpha + s), alpha != 0.0 ? alpha : 1.0);
        tau = (beta - alpha) / beta;
        const double sc = 1.0 / (alpha - beta);
        for (int i = lane; i < len; i += CTQR_WAVE) x[i] *= sc;
    }
    if (lane == 0) {
        *alpha_p = beta;
        *tau_out = tau;
    }
}

// S (c x c, LDS, ld LD) from tau and the Gram G = U^T U (LDS, ld LD) by the
// larft recurrence; S's strict lower part is zero.
__device__ inline void larft(const double *tau, const double *G, double *Sl, int c)
{
    for (int e = threadIdx.x; e < TB * TB; e += NT) Sl[(e / TB) * LD + e % TB] = 0.0;
    __syncthreads();
    for (int p = 0; p < c; ++p) {
        // S_{0:p, p} = -tau_p S_{0:p, 0:p} G_{0:p, p}
        if ((int)threadIdx.x < p) {
            const int a = threadIdx.x;
            double acc = 0.0;
            for (int q = a; q < p; ++q) acc += Sl[q * LD + a] * G[p * LD + q];
            Sl[p * LD + a] = -tau[p] * acc;
        }
        if (threadIdx.x == 0) Sl[p * LD + p] = tau[p];
        __syncthreads();
    }
}

__device__ inline void store_s(const double *Sl, double *g, int b)
{
    for (int e = threadIdx.x; e < b * b; e += NT) g[e] = Sl[(e / b) * LD + e % b];
}

__device__ inline void load_s(double *Sl, const double *g, int b)
{
    for (int e = threadIdx.x; e < TB * TB; e += NT) {
        const int q = e / TB, a = e % TB;
        Sl[q * LD + a] = (a < b && q < b) ? g[q * b + a] : 0.0;
    }
}

// ---- factorization tasks ----------------------------------------------------

__global__ __launch_bounds__(NT)
void dense_qr_kernel(const int4 *__restrict__ tasks, Dims d, double *A, int64_t lda, double *Sf)
{
    __shared__ double T[TB * LD], G[TB * LD];
    __shared__ double tau[TB];
    const int4 t = tasks[blockIdx.x];
    const int k = t.z;
    const int r = d.rows(k), c = d.cols(k), kc = min(r, c);
    double *Ag = tile_ptr(A, lda, d, k, k);
    load_tile(T, Ag, lda, r, c);
    __syncthreads();
    const int wave = threadIdx.x / CTQR_WAVE, lane = threadIdx.x % CTQR_WAVE;
    for (int p = 0; p < kc; ++p) {
        if (wave == 0) larfg_wave0(&T[p * LD + p], &T[p * LD + p + 1], r - p - 1, &tau[p]);
        __syncthreads();
        // columns q > p: w = T[p, q] + v^T T[p+1:, q]; T[p:, q] -= tau w [1; v]
        for (int q = p + 1 + wave; q < c; q += NT / CTQR_WAVE) {
            double s = 0.0;
            for (int i = p + 1 + lane; i < r; i += CTQR_WAVE) s += T[p * LD + i] * T[q * LD + i];
            const double tq = T[q * LD + p];
            const double w = tau[p] * (tq + wave_sum(s));
            if (lane == 0) T[q * LD + p] -= w;
            for (int i = p + 1 + lane; i < r; i += CTQR_WAVE) T[q * LD + i] -= w * T[p * LD + i];
        }
        __syncthreads();
    }
    // Gram of U (unit lower trapezoid r x kc)
    for (int e = threadIdx.x; e < kc * kc; e += NT) {
        const int a = e % kc, p = e / kc;
        double acc = 0.0;
        for (int i = 0; i < r; ++i) {
            const double ua = i < a ? 0.0 : (i == a ? 1.0 : T[a * LD + i]);
            const double up = i < p ? 0.0 : (i == p ? 1.0 : T[p * LD + i]);
            acc += ua * up;
        }
        G[p * LD + a] = acc;
    }
    __syncthreads();
    store_tile(T, Ag, lda, r, c);
    __syncthreads();
    larft(tau, G, T, kc);   // S reuses T's storage
    store_s(T, s_ptr(Sf, d, k, k), d.b);
}

__global__ __launch_bounds__(NT)
void td_qr_kernel(const int4 *__restrict__ tasks, Dims d, double *A, int64_t lda, double *Sf)
{
    __shared__ double R[TB * LD], D[TB * LD];
    __shared__ double tau[TB];
    const int4 t = tasks[blockIdx.x];
    const int i = t.y, k = t.z;
    const int c = d.cols(k), r = d.rows(i);
    double *Rg = tile_ptr(A, lda, d, k, k), *Dg = tile_ptr(A, lda, d, i, k);
    load_tile(R, Rg, lda, c, c);
    load_tile(D, Dg, lda, r, c);
    __syncthreads();
    const int wave = threadIdx.x / CTQR_WAVE, lane = threadIdx.x % CTQR_WAVE;
    for (int p = 0; p < c; ++p) {
        if (wave == 0) larfg_wave0(&R[p * LD + p], &D[p * LD], r, &tau[p]);
        __syncthreads();
        // columns q > p: w = R[p, q] + v^T D[:, q]; R[p, q] -= tau w; D[:, q] -= tau w v
        for (int q = p + 1 + wave; q < c; q += NT / CTQR_WAVE) {
            double s = 0.0;
            for (int e = lane; e < r; e += CTQR_WAVE) s += D[p * LD + e] * D[q * LD + e];
            const double rq = R[q * LD + p];
            const double w = tau[p] * (rq + wave_sum(s));
            if (lane == 0) R[q * LD + p] -= w;
            for (int e = lane; e < r; e += CTQR_WAVE) D[q * LD + e] -= w * D[p * LD + e];
        }
        __syncthreads();
    }
    // R back: the upper triangle only (the strict lower part of A_kk holds
    // dense_qr's reflectors)
    for (int e = threadIdx.x; e < c * c; e += NT) {
        const int q = e / c, a = e % c;
        if (a <= q) Rg[(int64_t)q * lda + a] = R[q * LD + a];
    }
    store_tile(D, Dg, lda, r, c);
    __syncthreads();
    // Gram of U = [I; D]: the identity part adds nothing off the diagonal
    for (int e = threadIdx.x; e < c * c; e += NT) {
        const int a = e % c, p = e / c;
        double acc = 0.0;
        for (int q = 0; q < r; ++q) acc += D[a * LD + q] * D[p * LD + q];
        R[p * LD + a] = acc;
    }
    __syncthreads();
    larft(tau, R, D, c);
    store_s(D, s_ptr(Sf, d, i, k), d.b);
}

// C <- (I - V S V^T)^T C: V the unit lower trapezoid (r x kc) of the block at
// Vg, S (kc x kc upper, column-major, ld b) at Sg, C (r x nc) at Cg.  The
// caller's LDS buffers V, Cl, W, Wt hold V, C, W = V^T C and W' = S^T W.
__device__ void apply_dense_dev(const double *Vg, int64_t ldv, const double *Sg, int b, int r, int kc, double *Cg,
                                int64_t ldc, int nc, double *V, double *Cl, double *W, double *Wt)
{
    load_tile(V, Vg, ldv, r, kc);
    load_tile(Cl, Cg, ldc, r, nc);
    __syncthreads();
    for (int e = threadIdx.x; e < kc * nc; e += NT) {
        const int a = e % kc, q = e / kc;
        double acc = Cl[q * LD + a];
        for (int i = a + 1; i < r; ++i) acc += V[a * LD + i] * Cl[q * LD + i];
        W[q * LD + a] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kc * nc; e += NT) {
        const int a = e % kc, q = e / kc;
        double acc = 0.0;
        for (int p = 0; p <= a; ++p) acc += Sg[a * b + p] * W[q * LD + p];
        Wt[q * LD + a] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < r * nc; e += NT) {
        const int i = e % r, q = e / r;
        double acc = Wt[q * LD + min(i, kc - 1)] * (i < kc ? 1.0 : 0.0);
        const int amax = min(i, kc) - 1;   // a < i and a < kc: V[i, a] below the diagonal
        for (int a = 0; a <= amax; ++a) acc += V[a * LD + i] * Wt[q * LD + a];
        Cg[(int64_t)q * ldc + i] = Cl[q * LD + i] - acc;
    }
}

// [F; G] <- (I - U S U^T)^T [F; G], U = [I; D]: D (r x kc) at Dg, S at Sg,
// F's first kc rows at Fg, G (r x nc) at Gg.
__device__ void apply_td_dev(const double *Dg, int64_t ldd, const double *Sg, int b, int r, int kc, double *Fg,
                             int64_t ldf, double *Gg, int64_t ldg, int nc, double *Dl, double *Gl, double *W,
                             double *Wt)
{
    load_tile(Dl, Dg, ldd, r, kc);
    load_tile(Gl, Gg, ldg, r, nc);
    __syncthreads();
    for (int e = threadIdx.x; e < kc * nc; e += NT) {
        const int a = e % kc, q = e / kc;
        double acc = Fg[(int64_t)q * ldf + a];
        for (int s2 = 0; s2 < r; ++s2) acc += Dl[a * LD + s2] * Gl[q * LD + s2];
        W[q * LD + a] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kc * nc; e += NT) {
        const int a = e % kc, q = e / kc;
        double acc = 0.0;
        for (int p = 0; p <= a; ++p) acc += Sg[a * b + p] * W[q * LD + p];
        Wt[q * LD + a] = acc;
    }
    __syncthreads();
    for (int e = threadIdx.x; e < kc * nc; e += NT) {
        const int a = e % kc, q = e / kc;
        Fg[(int64_t)q * ldf + a] -= Wt[q * LD + a];
    }
    for (int e = threadIdx.x; e < r * nc; e += NT) {
        const int s2 = e % r, q = e / r;
        double acc = 0.0;
        for (int a = 0; a < kc; ++a) acc += Dl[a * LD + s2] * Wt[q * LD + a];
        Gg[(int64_t)q * ldg + s2] = Gl[q * LD + s2] - acc;
    }
}

__global__ __launch_bounds__(NT)
void apply_dense_kernel(const int4 *__restrict__ tasks, Dims d, double *A, int64_t lda, const double *Sf)
{
    __shared__ double V[TB * LD], Cl[TB * LD], W[TB * LD], Wt[TB * LD];
    const int4 t = tasks[blockIdx.x];
    const int k = t.z, j = t.w;
    const int r = d.rows(k), kc = min(r, d.cols(k));
    apply_dense_dev(tile_ptr(A, lda, d, k, k), lda, s_ptr(const_cast<double *>(Sf), d, k, k), d.b, r, kc,
                    tile_ptr(A, lda, d, k, j), lda, d.cols(j), V, Cl, W, Wt);
}

__global__ __launch_bounds__(NT)
void apply_td_kernel(const int4 *__restrict__ tasks, Dims d, double *A, int64_t lda, const double *Sf)
{
    __shared__ double Dl[TB * LD], Gl[TB * LD], W[TB * LD], Wt[TB * LD];
    const int4 t = tasks[blockIdx.x];
    const int i = t.y, k = t.z, j = t.w;
    apply_td_dev(tile_ptr(A, lda, d, i, k), lda, s_ptr(const_cast<double *>(Sf), d, i, k), d.b, d.rows(i),
                 d.cols(k), tile_ptr(A, lda, d, k, j), lda, tile_ptr(A, lda, d, i, j), lda, d.cols(j), Dl, Gl, W,
                 Wt);
}

// ---- solve tasks: blockIdx.y is a chunk of RHS_CHUNK right-hand-side columns --

__global__ __launch_bounds__(NT)
void solve_apply_dense_kernel(const int4 *__restrict__ tasks, Dims d, const double *A, int64_t lda,
                              const double *Sf, double *B, int64_t ldb, int S)
{
    __shared__ double V[TB * LD], Cl[TB * LD], W[TB * LD], Wt[TB * LD];
    const int4 t = tasks[blockIdx.x];
    const int k = t.z, s0 = blockIdx.y * RHS_CHUNK;
    const int r = d.rows(k), kc = min(r, d.cols(k));
    double *Ac = const_cast<double *>(A);
    apply_dense_dev(tile_ptr(Ac, lda, d, k, k), lda, s_ptr(const_cast<double *>(Sf), d, k, k), d.b, r, kc,
                    B + (int64_t)s0 * ldb + (int64_t)k * d.b, ldb, min(RHS_CHUNK, S - s0), V, Cl, W, Wt);
}

__global__ __launch_bounds__(NT)
void solve_apply_td_kernel(const int4 *__restrict__ tasks, Dims d, const double *A, int64_t lda, const double *Sf,
                           double *B, int64_t ldb, int S)
{
    __shared__ double Dl[TB * LD], Gl[TB * LD], W[TB * LD], Wt[TB * LD];
    const int4 t = tasks[blockIdx.x];
    const int i = t.y, k = t.z, s0 = blockIdx.y * RHS_CHUNK;
    double *Ac = const_cast<double *>(A);
    double *Bc = B + (int64_t)s0 * ldb;
    apply_td_dev(tile_ptr(Ac, lda, d, i, k), lda, s_ptr(const_cast<double *>(Sf), d, i, k), d.b, d.rows(i),
                 d.cols(k), Bc + (int64_t)k * d.b, ldb, Bc + (int64_t)i * d.b, ldb, min(RHS_CHUNK, S - s0), Dl, Gl,
                 W, Wt);
}

// B_i -= R_ij X_j (rows of block row i of R: c_i; X_j: the first c_j rows of B_j)
__global__ __launch_bounds__(NT)
void solve_gemm_kernel(const int4 *__restrict__ tasks, Dims d, const double *A, int64_t lda, double *B,
                       int64_t ldb, int S)
{
    __shared__ double Rl[TB * LD], Xl[TB * LD];
    const int4 t = tasks[blockIdx.x];
    const int i = t.y, j = t.w, s0 = blockIdx.y * RHS_CHUNK, nc = min(RHS_CHUNK, S - s0);
    const int ci = d.cols(i), cj = d.cols(j);
    load_tile(Rl, tile_ptr(const_cast<double *>(A), lda, d, i, j), lda, ci, cj);
    double *Bc = B + (int64_t)s0 * ldb;
    load_tile(Xl, Bc + (int64_t)j * d.b, ldb, cj, nc);
    __syncthreads();
    for (int e = threadIdx.x; e < ci * nc; e += NT) {
        const int a = e % ci, q = e / ci;
        double acc = 0.0;
        for (int p = 0; p < cj; ++p) acc += Rl[p * LD + a] * Xl[q * LD + p];
        Bc[(int64_t)q * ldb + (int64_t)i * d.b + a] -= acc;
    }
}

// X_i = R_ii^-1 B_i: one thread per right-hand side, back substitution over
// the block's c_i rows (R_ii in LDS)
__global__ __launch_bounds__(NT)
void solve_trsm_kernel(const int4 *__restrict__ tasks, Dims d, const double *A, int64_t lda, double *B, int64_t ldb,
                       int S)
{
    __shared__ double Rl[TB * LD], Xl[TB * LD];
    const int4 t = tasks[blockIdx.x];
    const int i = t.y, s0 = blockIdx.y * RHS_CHUNK, nc = min(RHS_CHUNK, S - s0);
    const int c = d.cols(i);
    load_tile(Rl, tile_ptr(const_cast<double *>(A), lda, d, i, i), lda, c, c);
    double *Bc = B + (int64_t)s0 * ldb + (int64_t)i * d.b;
    load_tile(Xl, Bc, ldb, c, nc);
    __syncthreads();
    const int q = threadIdx.x;
    if (q < nc) {
        for (int p = c - 1; p >= 0; --p) {
            double acc = Xl[q * LD + p];
            for (int a = p + 1; a < c; ++a) acc -= Rl[a * LD + p] * Xl[q * LD + a];
            Xl[q * LD + p] = acc / Rl[p * LD + p];
        }
    }
    __syncthreads();
    store_tile(Xl, Bc, ldb, c, nc);
}

}  // namespace

// ---- host side ----------------------------------------------------------------

// Task lists in the order of the paper's task tables (int4: type, i, k, j).
std::vector<int4> tile_qr_tasks(int mt, int nt)
{
    std::vector<int4> out;
    for (int j = 0; j < nt; ++j) {
        for (int k = 0; k < std::min(j, mt); ++k) {
            out.push_back(make_int4(CTQR_TASK_APPLY_DENSE, k, k, j));
            for (int i = k + 1; i < mt; ++i) out.push_back(make_int4(CTQR_TASK_APPLY_TD, i, k, j));
        }
        if (j < mt) {
            out.push_back(make_int4(CTQR_TASK_DENSE_QR, j, j, j));
            for (int i = j + 1; i < mt; ++i) out.push_back(make_int4(CTQR_TASK_TD_QR, i, j, j));
        }
    }
    return out;
}

std::vector<int4> tile_solve_tasks(int mt, int nt)
{
    std::vector<int4> out;
    for (int k = 0; k < std::min(mt, nt); ++k) {
        out.push_back(make_int4(CTQR_TASK_APPLY_DENSE, k, k, -1));
        for (int i = k + 1; i < mt; ++i) out.push_back(make_int4(CTQR_TASK_APPLY_TD, i, k, -1));
    }
    for (int i = nt - 1; i >= 0; --i) {
        for (int j = i + 1; j < nt; ++j) out.push_back(make_int4(CTQR_TASK_GEMM, i, i, j));
        out.push_back(make_int4(CTQR_TASK_TRSM, i, i, i));
    }
    return out;
}

namespace {

// Resources a task reads and writes, as integer ids: block (i, j) of A as
// 2 (i nt + j) (its upper triangle and the rest as two ids for the diagonal
// blocks: 2 id for the strict lower part, 2 id + 1 for the upper triangle;
// off-diagonal blocks use 2 id), the S factor (i, k) as base_s + i nt + k,
// block row i of B as base_b + i.
struct Access {
    int n = 0;
    int64_t id[8];
    bool w[8];
    void add(int64_t r, bool write) { id[n] = r; w[n++] = write; }
};

Access access_of(const int4 &t, int mt, int nt, bool solve)
{
    const int64_t nb = (int64_t)mt * nt;
    auto blk = [&](int i, int j) { return 2 * ((int64_t)i * nt + j); };
    auto up = [&](int i) { return blk(i, i) + 1; };
    auto sf = [&](int i, int k) { return 2 * nb + (int64_t)i * nt + k; };
    auto brow = [&](int i) { return 3 * nb + i; };
    Access a;
    const int i = t.y, k = t.z, j = t.w;
    switch (t.x) {
    case CTQR_TASK_DENSE_QR:
        a.add(blk(k, k), true); a.add(up(k), true); a.add(sf(k, k), true);
        break;
    case CTQR_TASK_TD_QR:
        a.add(up(k), true); a.add(blk(i, k), true); a.add(sf(i, k), true);
        break;
    case CTQR_TASK_APPLY_DENSE:
        a.add(blk(k, k), false); a.add(sf(k, k), false);
        if (solve) a.add(brow(k), true);
        else { a.add(blk(k, j), true); if (j == k) a.add(up(k), true); }
        break;
    case CTQR_TASK_APPLY_TD:
        a.add(blk(i, k), false); a.add(sf(i, k), false);
        if (solve) { a.add(brow(k), true); a.add(brow(i), true); }
        else { a.add(blk(k, j), true); a.add(blk(i, j), true); }
        break;
    case CTQR_TASK_GEMM:
        a.add(blk(i, j), false); a.add(brow(j), false); a.add(brow(i), true);
        break;
    default:   // CTQR_TASK_TRSM
        a.add(up(i), false); a.add(brow(i), true);
        break;
    }
    return a;
}

}  // namespace

// Dependency level of each task (0-based): one more than the latest level of
// a task whose writes it reads or whose reads or writes it overwrites.
std::vector<int> tile_levels(const std::vector<int4> &tasks, int mt, int nt, bool solve)
{
    std::unordered_map<int64_t, int> last_w, last_r;
    std::vector<int> lev(tasks.size());
    for (size_t q = 0; q < tasks.size(); ++q) {
        const Access a = access_of(tasks[q], mt, nt, solve);
        int L = 0;
        for (int e = 0; e < a.n; ++e) {
            auto it = last_w.find(a.id[e]);
            if (it != last_w.end()) L = std::max(L, it->second + 1);
            if (a.w[e]) {
                auto ir = last_r.find(a.id[e]);
                if (ir != last_r.end()) L = std::max(L, ir->second + 1);
            }
        }
        lev[q] = L;
        for (int e = 0; e < a.n; ++e) {
            if (a.w[e]) last_w[a.id[e]] = L;
            else last_r[a.id[e]] = std::max(last_r.count(a.id[e]) ? last_r[a.id[e]] : 0, L);
        }
    }
    return lev;
}

// Launch plan: tasks sorted by (level, type), stable, and the segments of
// equal (level, type).
struct TilePlan {
    std::vector<int4> tasks;
    std::vector<std::pair<size_t, size_t>> segs;   // [begin, end) in tasks
};

TilePlan tile_plan(const std::vector<int4> &tasks, int mt, int nt, bool solve)
{
    const std::vector<int> lev = tile_levels(tasks, mt, nt, solve);
    std::vector<size_t> order(tasks.size());
    for (size_t q = 0; q < order.size(); ++q) order[q] = q;
    std::stable_sort(order.begin(), order.end(), [&](size_t a, size_t b) {
        return lev[a] != lev[b] ? lev[a] < lev[b] : tasks[a].x < tasks[b].x;
    });
    TilePlan p;
    for (size_t q = 0; q < order.size(); ++q) {
        p.tasks.push_back(tasks[order[q]]);
        const bool start = q == 0 || lev[order[q]] != lev[order[q - 1]] || tasks[order[q]].x != tasks[order[q - 1]].x;
        if (start) p.segs.push_back({q, q + 1});
        else p.segs.back().second = q + 1;
    }
    return p;
}

ctqr_status tile_qr_run(int m, int n, int b, double *A, int64_t lda, double *Sf, int4 *dtasks, hipStream_t st)
{
    const int mt = (int)ceil_div(m, b), nt = (int)ceil_div(n, b);
    const TilePlan p = tile_plan(tile_qr_tasks(mt, nt), mt, nt, false);
    HIP_TRY(hipMemcpyAsync(dtasks, p.tasks.data(), p.tasks.size() * sizeof(int4), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));   // the host vector is freed on return
    const Dims d{m, n, b, mt, nt};
    for (auto &sg : p.segs) {
        const int4 *tk = dtasks + sg.first;
        const dim3 grid((unsigned)(sg.second - sg.first));
        switch (p.tasks[sg.first].x) {
        case CTQR_TASK_DENSE_QR: LAUNCH_TRY(dense_qr_kernel, grid, dim3(NT), 0, st, tk, d, A, lda, Sf); break;
        case CTQR_TASK_TD_QR: LAUNCH_TRY(td_qr_kernel, grid, dim3(NT), 0, st, tk, d, A, lda, Sf); break;
        case CTQR_TASK_APPLY_DENSE:
            LAUNCH_TRY(apply_dense_kernel, grid, dim3(NT), 0, st, tk, d, A, lda, (const double *)Sf);
            break;
        default: LAUNCH_TRY(apply_td_kernel, grid, dim3(NT), 0, st, tk, d, A, lda, (const double *)Sf); break;
        }
    }
    return CTQR_OK;
}

ctqr_status tile_solve_run(int m, int n, int b, const double *A, int64_t lda, const double *Sf, double *B,
                           int64_t ldb, int S, int4 *dtasks, hipStream_t st)
{
    const int mt = (int)ceil_div(m, b), nt = (int)ceil_div(n, b);
    const TilePlan p = tile_plan(tile_solve_tasks(mt, nt), mt, nt, true);
    HIP_TRY(hipMemcpyAsync(dtasks, p.tasks.data(), p.tasks.size() * sizeof(int4), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));
    const Dims d{m, n, b, mt, nt};
    const unsigned chunks = (unsigned)ceil_div(S, RHS_CHUNK);
    for (auto &sg : p.segs) {
        const int4 *tk = dtasks + sg.first;
        const dim3 grid((unsigned)(sg.second - sg.first), chunks);
        switch (p.tasks[sg.first].x) {
        case CTQR_TASK_APPLY_DENSE:
            LAUNCH_TRY(solve_apply_dense_kernel, grid, dim3(NT), 0, st, tk, d, A, lda, Sf, B, ldb, S);
            break;
        case CTQR_TASK_APPLY_TD:
            LAUNCH_TRY(solve_apply_td_kernel, grid, dim3(NT), 0, st, tk, d, A, lda, Sf, B, ldb, S);
            break;
        case CTQR_TASK_GEMM: LAUNCH_TRY(solve_gemm_kernel, grid, dim3(NT), 0, st, tk, d, A, lda, B, ldb, S); break;
        default: LAUNCH_TRY(solve_trsm_kernel, grid, dim3(NT), 0, st, tk, d, A, lda, B, ldb, S); break;
        }
    }
    return CTQR_OK;
}
