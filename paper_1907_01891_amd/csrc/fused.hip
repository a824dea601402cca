// Persistent solve kernels for few right-hand sides (S <= FUSED_MAX_S).
//
// With a handful of slices, the block-at-a-time chains of the wide solve
// (three GEMM launches per block reflector, two per diagonal block of the
// substitutions) are bound by launch and ramp-up latency, not by the one
// pass over the factor that the work needs.  These kernels run a whole phase
// as one cooperative launch of one workgroup per compute unit, ordered by
// grid barriers (common.h), with the same arithmetic per block:
//
//   trsm_fused<T, false>: R X = C, block rows from the bottom (Section II-C,
//       "System solving": Trsm_lunn on the diagonal block, Gemm_nn_mo for the
//       rows above), X_i = inv(R_ii) C_i; C_{0:r0} -= R_{0:r0, i} X_i;
//   trsm_fused<T, true>: R^T Y = C, block rows from the top,
//       Y_i = inv(R_ii)^T C_i; C_{i+1:} -= R_{i, i+1:}^T Y_i;
//   qtb_fused<T>: Q^T B over the block reflectors (Eq. 4), block k:
//       W = V_k^T B;  W' = T_k^T W;  B -= V_k W'.
//
// Rows of the right-hand side are owned in 64-row chunks, chunk c by
// workgroup c mod G, and stay in LDS for the whole launch; only the small
// per-step vectors (a diagonal block's right-hand side, its solution, the
// per-workgroup partial products of V_k^T B and W') cross workgroups, through
// agent-coherent stores and loads.  The factor streams through LDS in tiles
// of 64 rows x 128 inner indices, the next tile loaded while the current one
// is used; the four waves of a workgroup split each tile's inner indices (or
// rows), every thread keeping all slices of its row (column), and their
// partial sums are added in wave order.  Every sum is taken in a fixed order
// that does not depend on the number of slices or on timing, so the results
// are reproducible and a slice's result does not depend on the others.
#include <algorithm>
#include <mutex>

#include "common.h"
#include "kernels.h"

namespace {

constexpr int FNT = 256;                 // threads per workgroup
constexpr int NW = FNT / 64;             // waves per workgroup
constexpr int CH = 64;                   // rows per ownership chunk
constexpr int BIG = TRSM_BIG;            // diagonal block of the substitutions
constexpr int TBK = 64;                  // inner-dimension depth of a staged tile
constexpr int XCH = 256;                 // rows of a staged per-step vector block
constexpr int SM = FUSED_MAX_S;          // slice capacity
constexpr int RT_ELEMS = TBK * (CH + 1); // staged tile (also the partial sums' room)

static_assert(SM % 4 == 0 && SM <= 16, "slices in groups of four");
static_assert(XCH == FNT, "one staged row per thread");
static_assert(NW * CH * SM <= RT_ELEMS && NW * TBK * SM <= RT_ELEMS, "partial sums fit the tile's room");
static_assert(XCH % TBK == 0 && CH % NW == 0 && TBK % NW == 0, "tiles split evenly");

template <typename T>
__device__ __attribute__((always_inline)) inline void st_coh(T *p, T v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
template <typename T>
__device__ __attribute__((always_inline)) inline T ld_coh(const T *p)
{
    return __hip_atomic_load(const_cast<T *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// sum over the 32 lanes of a half wave, in a fixed butterfly order
template <typename T>
__device__ __attribute__((always_inline)) inline T half_wave_sum(T v)
{
#pragma unroll
    for (int o = 16; o > 0; o >>= 1) v += __shfl_xor(v, o, 32);
    return v;
}

// LDS: owned chunks Cl[q][rho][SM], a staged vector block (Xs[b][SM] for the
// chunk updates, Xs[s][XCH] for the diagonal-block products), a staged tile
// Rt[TBK][CH + 1].
template <typename T>
struct Lds {
    T *Cl, *Xs, *Rt;
    __device__ Lds(unsigned char *raw, int qmax)
    {
        Cl = (T *)raw;
        Xs = Cl + (size_t)qmax * CH * SM;
        Rt = Xs + SM * XCH;
    }
};

}  // namespace

size_t fused_lds_bytes(int qmax, size_t esz)
{
    return ((size_t)qmax * CH * SM + SM * XCH + RT_ELEMS) * esz;
}

namespace {

// Staged tiles A[rho, bb], rho < CH rows of a chunk starting at row c0,
// bb < TBK inner indices from b0, kept in LDS as Rt[bb][rho]:
//   TILE_R:  A = R[c0 + rho, b0 + bb] (column-major reads along rho);
//   TILE_RT: A = R[b0 + bb, c0 + rho] (reads along bb);
//   TILE_V:  A = V[c0 + rho, b0 + bb], the Householder vectors stored below
//            the diagonal of the factor: one on the diagonal, zero above it.
// Entries outside the nrow x ncol matrix are zero.
enum { TILE_R = 0, TILE_RT = 1, TILE_V = 2 };
constexpr int TPT = TBK * CH / FNT;   // tile entries per thread

// entry k of thread t: consecutive lanes take consecutive addresses (rho for
// the column-major reads, bb for the transposed ones)
template <int MODE>
__device__ __attribute__((always_inline)) inline void tile_entry(int t, int k, int &rho, int &bb)
{
    if (MODE == TILE_RT) {
        bb = t % TBK;
        rho = t / TBK + (FNT / TBK) * k;
    } else {
        rho = t % CH;
        bb = t / CH + (FNT / CH) * k;
    }
}

template <typename T, int MODE>
__device__ __attribute__((always_inline)) inline void load_tile(const T *__restrict__ R, int64_t ldr, int nrow, int ncol, int c0, int b0,
                                 T (&reg)[TPT])
{
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        int rho, bb;
        tile_entry<MODE>(t, k, rho, bb);
        const int gi = MODE == TILE_RT ? b0 + bb : c0 + rho;    // A = R[gi, gj]
        const int gj = MODE == TILE_RT ? c0 + rho : b0 + bb;
        const bool ok = gi < nrow && gj < ncol;
        T v = ok ? R[(int64_t)gj * ldr + gi] : T(0);
        if (MODE == TILE_V) v = gi > gj ? v : (gi == gj && ok ? T(1) : T(0));
        reg[k] = v;
    }
}

template <typename T, int MODE>
__device__ __attribute__((always_inline)) inline void store_tile(T *Rt, const T (&reg)[TPT])
{
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < TPT; ++k) {
        int rho, bb;
        tile_entry<MODE>(t, k, rho, bb);
        Rt[bb * (CH + 1) + rho] = reg[k];
    }
}

// Stage rows 0 .. nbb of an S-column block (column s at src + s lds) into
// LDS through agent-coherent loads, all of a thread's loads issued before any
// is used (thread t takes row t of every column): ROWS true gives Xs[b][SM]
// (a row's slices together), false Xs[s][XCH].  Rows past nbb are zero.
template <typename T, bool ROWS>
__device__ __attribute__((always_inline)) inline void stage_coh(T *Xs, const T *src, int64_t lds, int nbb, int S)
{
    const int t = threadIdx.x;
    T v[SM];
#pragma unroll
    for (int s = 0; s < SM; ++s) v[s] = (s < S && t < nbb) ? ld_coh(&src[(int64_t)s * lds + t]) : T(0);
#pragma unroll
    for (int s = 0; s < SM; ++s) Xs[ROWS ? t * SM + s : s * XCH + t] = v[s];
}

// acc[s] += a x[s] for the first 4 NG slices (x: consecutive values; the
// slices past S are zero in LDS).  NG is a compile-time count, so the loop
// has no branches and its LDS reads can be issued ahead of the products.
template <int NG, typename T>
__device__ __attribute__((always_inline)) inline void axpy_slices(T (&acc)[SM], T a, const T *x)
{
#pragma unroll
    for (int s = 0; s < 4 * NG; ++s) acc[s] += a * x[s];
}

// Tiles stream through LDS with NP of them in flight (registers): tile it is
// item(it) -> (c0, b0).  prime() requests tiles 0 .. NP-1 (it may run early,
// e.g. before a grid barrier, since the factor is read only); run() stores
// each tile into Rt, requests tile it + NP into the freed registers and calls
// body(it).  count and the items are the same for every thread.
template <typename T>
constexpr int ring_depth()
{
    return sizeof(T) == 4 ? 8 : 4;             // 128 registers of tiles in flight
}

template <typename T, int MODE>
struct TileStream {
    static constexpr int NP = ring_depth<T>();
    T ring[NP][TPT];
    template <typename Item>
    __device__ __attribute__((always_inline)) void prime(const T *R, int64_t ldr, int nrow, int ncol, int count, Item item)
    {
#pragma unroll
        for (int u = 0; u < NP; ++u)
            if (u < count) {
                int c0, b0;
                item(u, c0, b0);
                load_tile<T, MODE>(R, ldr, nrow, ncol, c0, b0, ring[u]);
            }
    }
    template <typename Item, typename Body>
    __device__ __attribute__((always_inline)) void run(const T *R, int64_t ldr, int nrow, int ncol, int count, Item item, Body body, T *Rt)
    {
        for (int it0 = 0; it0 < count; it0 += NP) {
#pragma unroll
            for (int u = 0; u < NP; ++u) {
                const int it = it0 + u;
                if (it < count) {
                    __syncthreads();           // the previous tile (or partial sums) has been read
                    store_tile<T, MODE>(Rt, ring[u]);
                    __syncthreads();
                    if (it + NP < count) {
                        int c0, b0;
                        item(it + NP, c0, b0);
                        load_tile<T, MODE>(R, ldr, nrow, ncol, c0, b0, ring[u]);
                    }
                    body(it);
                }
            }
        }
    }
};

// acc += Rt-tile x Xs rows xb0 .. xb0 + TBK for thread (rho = t % 64, wave
// g): inner indices g*TBK/NW .. of the tile, in order, all slices
template <int NG, typename T>
__device__ __attribute__((always_inline)) inline void tile_axpy(T (&acc)[SM], const Lds<T> &L, int xb0)
{
    constexpr int QB = TBK / NW;
    const int rho = threadIdx.x % 64, g = threadIdx.x / 64;
#pragma unroll
    for (int k = 0; k < QB; ++k) {
        const int bb = g * QB + k;
        axpy_slices<NG>(acc, L.Rt[bb * (CH + 1) + rho], L.Xs + (xb0 + bb) * SM);
    }
}

// Clq -= the sum over the waves of acc (in wave order), through Rt; acc is
// cleared.  Called by every thread after its last tile_axpy of the chunk.
template <typename T>
__device__ __attribute__((always_inline)) inline void chunk_flush(T (&acc)[SM], const Lds<T> &L, T *Clq, int S)
{
    const int t = threadIdx.x, rho = t % 64, g = t / 64;
    __syncthreads();
    T *red = L.Rt;                             // [g][rho][SM]
#pragma unroll
    for (int s = 0; s < SM; ++s) {
        red[(g * CH + rho) * SM + s] = acc[s];
        acc[s] = T(0);
    }
    __syncthreads();
    for (int e = t; e < CH * SM; e += FNT) {
        const int r = e / SM, s = e % SM;
        if (s < S) {
            T v = red[r * SM + s];
#pragma unroll
            for (int u = 1; u < NW; ++u) v += red[(u * CH + r) * SM + s];
            Clq[r * SM + s] -= v;
        }
    }
}

// row a of a half wave's diagonal-block product, lane l: entries
// b0 + l + 32 i of the row (zero past bw)
template <typename T>
__device__ __attribute__((always_inline)) inline void load_mrow(T (&mv)[XCH / 32], const T *Mrow, int b0, int bw, bool have, int l)
{
#pragma unroll
    for (int i = 0; i < XCH / 32; ++i) {
        const int bb = b0 + l + 32 * i;
        mv[i] = (have && bb < bw) ? Mrow[bb] : T(0);
    }
}

// The block substitutions.  M holds the per-row data of the diagonal-block
// products: row a of inv(R_ii) (TRANS false) or of inv(R_ii)^T (TRANS true),
// contiguous, at M + (r0 + a) BIG.  E: BIG x SM exchange block (column s at
// E + s BIG).  X is written once per row, by the workgroup that computes it.
template <typename T, bool TRANS, int NG>
__global__ __launch_bounds__(FNT) void trsm_fused_kernel(int n, int S, const T *__restrict__ R, int64_t ldr,
                                                         const T *__restrict__ M, const T *__restrict__ C,
                                                         int64_t ldc, T *X, int64_t ldx, T *E, unsigned *bar,
                                                         const int *skip, ctqr_info *info)
{
    if (skip && *skip) return;                 // read by every workgroup before any barrier
    extern __shared__ __align__(16) unsigned char fused_lds[];
    const int G = gridDim.x, w = blockIdx.x, t = threadIdx.x;
    const int nch = (n + CH - 1) / CH, qmax = (nch + G - 1) / G;
    Lds<T> L(fused_lds, qmax);
    for (int q = 0; q < qmax; ++q) {
        const int c = w + q * G;
        if (c >= nch) break;
        for (int e = t; e < CH * SM; e += FNT) {
            const int rho = e / SM, s = e % SM, row = c * CH + rho;
            L.Cl[(q * CH + rho) * SM + s] = row < n && s < S ? C[(int64_t)s * ldc + row] : T(0);
        }
    }
    __syncthreads();
    unsigned epoch = 0;
    const int nblk = (n + BIG - 1) / BIG;
    TileStream<T, TRANS ? TILE_RT : TILE_R> ts;
    for (int step = 0; step < nblk; ++step) {
        const int i = TRANS ? step : nblk - 1 - step;
        const int r0 = i * BIG, bw = min(BIG, n - r0);
        // this step's chunk updates (c): chunks q in [qlo, qhi), items in the
        // order (block of XCH inner indices, chunk, tile); their first tiles
        // are requested now and arrive during (a) and (b)
        int qa = 0, qb = 0, qend = 0;
        for (int q = 0; q < qmax; ++q) {
            const int c = w + q * G;
            if (c >= nch) break;
            qend = q + 1;
            if (c * CH < r0) qa = q + 1;
            if (c * CH < r0 + bw) qb = q + 1;
        }
        const int qlo = TRANS ? qb : 0, qhi = TRANS ? qend : qa;
        constexpr int TPX = XCH / TBK;
        const int nxb = (bw + XCH - 1) / XCH, per_xb = (qhi - qlo) * TPX;
        const int cnt = step + 1 == nblk ? 0 : nxb * per_xb;
        auto item = [&](int it, int &c0, int &b0) {
            const int xb = it / per_xb, rem = it % per_xb;
            c0 = (w + (qlo + rem / TPX) * G) * CH;
            b0 = r0 + xb * XCH + (rem % TPX) * TBK;
        };
        ts.prime(R, ldr, n, n, cnt, item);
        // (a) the final right-hand side of block i into E
        for (int q = 0; q < qmax; ++q) {
            const int c = w + q * G;
            if (c >= nch) break;
            const int cr = c * CH;
            if (cr < r0 || cr >= r0 + bw) continue;
            for (int e = t; e < CH * S; e += FNT) {
                const int rho = e % CH, s = e / CH;
                if (cr + rho < n) st_coh(&E[(int64_t)s * BIG + cr + rho - r0], L.Cl[(q * CH + rho) * SM + s]);
            }
        }
        if (!grid_barrier(bar, epoch, info)) return;
        // (b) rows a = w + G (rl + 8 p) of the block's solution: each half wave
        // takes one row, its lanes stride the inner index, the lane sums are
        // combined by a fixed butterfly; the next block of the row is loaded
        // while the current one is used
        {
            const int rl = t / 32, l = t % 32;
            const int rows_here = bw > w ? (bw - w + G - 1) / G : 0;
            for (int p0 = 0; p0 < rows_here; p0 += FNT / 32) {
                const int a = w + G * (p0 + rl);
                const bool have = p0 + rl < rows_here;
                const T *Mrow = M + (int64_t)(r0 + (have ? a : 0)) * BIG;
                T acc[SM];
#pragma unroll
                for (int s = 0; s < SM; ++s) acc[s] = T(0);
                T mv[XCH / 32], mn[XCH / 32];
                load_mrow(mv, Mrow, 0, bw, have, l);
                for (int b0 = 0; b0 < bw; b0 += XCH) {
                    const int nbb = min(XCH, bw - b0);
                    __syncthreads();
                    stage_coh<T, false>(L.Xs, E + b0, BIG, nbb, S);
                    __syncthreads();
                    if (b0 + XCH < bw) load_mrow(mn, Mrow, b0 + XCH, bw, have, l);
#pragma unroll
                    for (int k = 0; k < XCH / 32; ++k) {
                        const int bb = l + 32 * k;
#pragma unroll
                        for (int s = 0; s < SM; ++s)
                            if (s < 4 * NG) acc[s] += mv[k] * L.Xs[s * XCH + bb];
                    }
#pragma unroll
                    for (int k = 0; k < XCH / 32; ++k) mv[k] = mn[k];
                }
#pragma unroll
                for (int s = 0; s < SM; ++s) acc[s] = half_wave_sum(acc[s]);
                if (have && l == 0)
                    for (int s = 0; s < S; ++s) st_coh(&X[(int64_t)s * ldx + r0 + a], acc[s]);
            }
        }
        if (step + 1 == nblk) break;           // nothing left to update
        // (c) the owned chunks outside block i that still take its update:
        // rows above it (TRANS false) or below it (TRANS true), qlo .. qhi;
        // their tiles were requested at the start of the step
        if (!grid_barrier(bar, epoch, info)) return;
        if (cnt == 0) continue;
        T acc[SM];
#pragma unroll
        for (int s = 0; s < SM; ++s) acc[s] = T(0);
        ts.run(R, ldr, n, n, cnt, item, [&](int it) {
            const int xb = it / per_xb, rem = it % per_xb, q = qlo + rem / TPX, bt = (rem % TPX) * TBK;
            if (rem == 0) {                    // a new block of X_i rows into Xs
                __syncthreads();
                stage_coh<T, true>(L.Xs, X + r0 + xb * XCH, ldx, min(XCH, bw - xb * XCH), S);
                __syncthreads();
            }
            tile_axpy<NG>(acc, L, bt);
            if (bt + TBK == XCH) chunk_flush(acc, L, L.Cl + (size_t)q * CH * SM, S);
        }, L.Rt);
        __syncthreads();
    }
}

// Q^T B over the block reflectors of width nb (<= 256): the rows of B
// (FP64, m x S) are read into LDS in the factor's precision, every block is
// applied, and the first n rows of the result go to Y (column-major, ldy).
// P: G x SM x nb per-workgroup partials of V_k^T B; Wv, Wt: SM x nb (W and
// W' of the block, slice s at s nb), all exchanged through agent-coherent
// accesses.
template <typename T, int NG>
__global__ __launch_bounds__(FNT) void qtb_fused_kernel(int m, int n, int nb, int S, const T *__restrict__ QR,
                                                        int64_t lda, const T *__restrict__ Tf,
                                                        const double *__restrict__ B, int64_t ldb, T *Y, int64_t ldy,
                                                        T *P, T *Wv, T *Wt, unsigned *bar, ctqr_info *info)
{
    extern __shared__ __align__(16) unsigned char fused_lds[];
    const int G = gridDim.x, w = blockIdx.x, t = threadIdx.x;
    const int nch = (m + CH - 1) / CH, qmax = (nch + G - 1) / G;
    Lds<T> L(fused_lds, qmax);
    for (int q = 0; q < qmax; ++q) {
        const int c = w + q * G;
        if (c >= nch) break;
        for (int e = t; e < CH * SM; e += FNT) {
            const int rho = e / SM, s = e % SM, row = c * CH + rho;
            L.Cl[(q * CH + rho) * SM + s] = row < m && s < S ? (T)B[(int64_t)s * ldb + row] : T(0);
        }
    }
    __syncthreads();
    unsigned epoch = 0;
    // chunks q < qlo lie above row k0; the first V tile of each block is
    // requested while the previous block's last tiles are used
    auto first_chunk = [&](int k0) {
        int qlo = 0;
        for (int q = 0; q < qmax; ++q) {
            const int c = w + q * G;
            if (c >= nch) break;
            if (c * CH < k0) qlo = q + 1;
        }
        return qlo;
    };
    int qend = 0;
    for (int q = 0; q < qmax; ++q)
        if (w + q * G < nch) qend = q + 1;
    TileStream<T, TILE_V> ts;
    // phase (1) items of block k0: (column tile, chunk); phase (4): (chunk, tile)
    int qlo = first_chunk(0), nq = qend - qlo, ntile = (min(nb, n) + TBK - 1) / TBK;
    auto item1 = [&](int it, int &c0, int &b0, int k0) {
        c0 = (w + (qlo + it % nq) * G) * CH;
        b0 = k0 + (it / nq) * TBK;
    };
    auto item4 = [&](int it, int &c0, int &b0, int k0) {
        c0 = (w + (qlo + it / ntile) * G) * CH;
        b0 = k0 + (it % ntile) * TBK;
    };
    ts.prime(QR, lda, m, n, ntile * nq, [&](int it, int &c0, int &b0) { item1(it, c0, b0, 0); });
    for (int k0 = 0; k0 < n; k0 += nb) {
        const int nbk = min(nb, n - k0);
        qlo = first_chunk(k0);
        nq = qend - qlo;
        ntile = (nbk + TBK - 1) / TBK;
        const int count = ntile * nq;
        auto it1 = [&](int it, int &c0, int &b0) { item1(it, c0, b0, k0); };
        auto it4 = [&](int it, int &c0, int &b0) { item4(it, c0, b0, k0); };
        // (1) this workgroup's partial V_k^T B over its chunks at or below row
        // k0 (nb is a multiple of CH, so a chunk lies wholly on one side), TBK
        // reflector columns at a time: thread (jj, h) takes column jj of the
        // tile, rows h*16 .. h*16 + 15 of each chunk in order, all slices; the
        // four quarters are added in order at the column tile's end.  The
        // tiles were requested at the end of the previous block.
        {
            const int jj = t % TBK, h = t / TBK;
            constexpr int QR4 = CH / NW;
            T acc[SM];
#pragma unroll
            for (int s = 0; s < SM; ++s) acc[s] = T(0);
            if (count == 0) {
                for (int e = t; e < nbk * S; e += FNT)
                    st_coh(&P[((int64_t)w * SM + e / nbk) * nb + e % nbk], T(0));
            }
            ts.run(QR, lda, m, n, count, it1, [&](int it) {
                const int jt = (it / nq) * TBK, q = qlo + it % nq;
                const T *Cq = L.Cl + (size_t)q * CH * SM;
#pragma unroll
                for (int k = 0; k < QR4; ++k) {
                    const int rho = h * QR4 + k;
                    axpy_slices<NG>(acc, L.Rt[jj * (CH + 1) + rho], Cq + rho * SM);
                }
                if (q + 1 == qend) {           // the column tile's last chunk: add the quarters
                    __syncthreads();
                    T *red = L.Rt;             // [h][jj][SM]
#pragma unroll
                    for (int s = 0; s < SM; ++s) {
                        red[(h * TBK + jj) * SM + s] = acc[s];
                        acc[s] = T(0);
                    }
                    __syncthreads();
                    for (int e = t; e < TBK * SM; e += FNT) {
                        const int j = e / SM, s = e % SM;
                        if (s < S && jt + j < nbk) {
                            T v = red[j * SM + s];
#pragma unroll
                            for (int u = 1; u < NW; ++u) v += red[(u * TBK + j) * SM + s];
                            st_coh(&P[((int64_t)w * SM + s) * nb + jt + j], v);
                        }
                    }
                }
            }, L.Rt);
        }
        // phase (4)'s tiles arrive during the barriers and exchanges
        ts.prime(QR, lda, m, n, count, it4);
        if (!grid_barrier(bar, epoch, info)) return;
        // (2) W = sum of the partials in workgroup order: entry e = (slice,
        // column) per half wave, lanes stride the workgroups (loads first)
        {
            const int hw = t / 32, l = t % 32, nent = nbk * S;
            constexpr int PU = 8;              // partials per lane and round (256 workgroups)
            for (int e0 = w * (FNT / 32); e0 < nent; e0 += G * (FNT / 32)) {
                const int e = e0 + hw, s = e / nbk, j = e % nbk;
                T v = T(0);
                for (int u0 = 0; u0 < G; u0 += 32 * PU) {
                    T pv[PU];
#pragma unroll
                    for (int i = 0; i < PU; ++i) {
                        const int u = u0 + l + 32 * i;
                        pv[i] = (e < nent && u < G) ? ld_coh(&P[((int64_t)u * SM + s) * nb + j]) : T(0);
                    }
#pragma unroll
                    for (int i = 0; i < PU; ++i) v += pv[i];
                }
                v = half_wave_sum(v);
                if (e < nent && l == 0) st_coh(&Wv[s * nb + j], v);
            }
        }
        if (!grid_barrier(bar, epoch, info)) return;
        // (3) W' = T_k^T W: W'[i, s] = sum_{u <= i} T[u, i] W[u, s]
        {
            const int hw = t / 32, l = t % 32, nent = nbk * S;
            const T *Tk = Tf + (int64_t)k0 * nb;
            constexpr int TU = 256 / 32;       // nb <= 256
            for (int e0 = w * (FNT / 32); e0 < nent; e0 += G * (FNT / 32)) {
                const int e = e0 + hw, s = e / nbk, i = e % nbk;
                T tv[TU], wv[TU];
#pragma unroll
                for (int k = 0; k < TU; ++k) {
                    const int u = l + 32 * k;
                    const bool ok = e < nent && u <= i;
                    tv[k] = ok ? Tk[(int64_t)i * nb + u] : T(0);
                    wv[k] = ok ? ld_coh(&Wv[s * nb + u]) : T(0);
                }
                T v = T(0);
#pragma unroll
                for (int k = 0; k < TU; ++k) v += tv[k] * wv[k];
                v = half_wave_sum(v);
                if (e < nent && l == 0) st_coh(&Wt[s * nb + i], v);
            }
        }
        if (!grid_barrier(bar, epoch, info)) return;
        // (4) B -= V_k W' on the owned chunks at or below row k0
        __syncthreads();
        stage_coh<T, true>(L.Xs, Wt, nb, nbk, S);
        __syncthreads();
        {
            T acc[SM];
#pragma unroll
            for (int s = 0; s < SM; ++s) acc[s] = T(0);
            ts.run(QR, lda, m, n, count, it4, [&](int it) {
                const int q = qlo + it / ntile, bt = (it % ntile) * TBK;
                tile_axpy<NG>(acc, L, bt);
                if (bt + TBK >= nbk) chunk_flush(acc, L, L.Cl + (size_t)q * CH * SM, S);
            }, L.Rt);
        }
        __syncthreads();
        // the next block's phase (1) tiles
        if (k0 + nb < n) {
            const int k1 = k0 + nb, nbk1 = min(nb, n - k1);
            qlo = first_chunk(k1);
            nq = qend - qlo;
            ntile = (nbk1 + TBK - 1) / TBK;
            ts.prime(QR, lda, m, n, ntile * nq, [&](int it, int &c0, int &b0) { item1(it, c0, b0, k1); });
        }
    }
    // the first n rows of Q^T B
    for (int q = 0; q < qmax; ++q) {
        const int c = w + q * G;
        if (c >= nch) break;
        for (int e = t; e < CH * S; e += FNT) {
            const int rho = e % CH, s = e / CH, row = c * CH + rho;
            if (row < n) Y[(int64_t)s * ldy + row] = L.Cl[(q * CH + rho) * SM + s];
        }
    }
}

}  // namespace

// the kernel instance of S slices: groups of four slices, 1, 2 or 4 of them
int slice_groups(int S) { return S <= 4 ? 1 : S <= 8 ? 2 : 4; }

template <typename T, bool TRANS>
const void *trsm_fn(int S)
{
    const int g = slice_groups(S);
    return g == 1 ? (const void *)trsm_fused_kernel<T, TRANS, 1>
                  : g == 2 ? (const void *)trsm_fused_kernel<T, TRANS, 2> : (const void *)trsm_fused_kernel<T, TRANS, 4>;
}

template <typename T>
const void *qtb_fn(int S)
{
    const int g = slice_groups(S);
    return g == 1 ? (const void *)qtb_fused_kernel<T, 1>
                  : g == 2 ? (const void *)qtb_fused_kernel<T, 2> : (const void *)qtb_fused_kernel<T, 4>;
}

int fused_grid()
{
    static int g = 0;
    if (!g) {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            g = p.multiProcessorCount;
        if (g < 1) g = 1;
    }
    return g;
}

ctqr_status fused_setup_once()
{
    const int l = (int)FUSED_MAX_LDS;
    for (int S : {1, 8, 16}) {
        for (const void *fn : {trsm_fn<float, false>(S), trsm_fn<float, true>(S), trsm_fn<double, false>(S),
                               trsm_fn<double, true>(S), qtb_fn<float>(S), qtb_fn<double>(S)})
            HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, l));
    }
    return CTQR_OK;
}

ctqr_status fused_setup_once();

// the kernels' dynamic LDS limit, once per process
ctqr_status fused_setup()
{
    static std::once_flag once;
    static ctqr_status st = CTQR_OK;
    std::call_once(once, [] { st = fused_setup_once(); });
    return st;
}

bool fused_fits(int64_t rows, size_t esz)
{
    const int G = fused_grid();
    const int64_t nch = ceil_div(rows, CH), qmax = ceil_div(nch, G);
    return fused_lds_bytes((int)qmax, esz) <= FUSED_MAX_LDS;
}

template <typename T>
ctqr_status trsm_fused(int n, int S, bool trans, const T *R, int64_t ldr, const T *Rinv, const T *C, int64_t ldc,
                       T *X, int64_t ldx, T *E, unsigned *bar, const int *skip, ctqr_info *info, hipStream_t st)
{
    if (S < 1 || S > SM || !fused_fits(n, sizeof(T))) return CTQR_EUNSUPPORTED;
    const int G = fused_grid();
    const int qmax = (int)ceil_div(ceil_div(n, CH), G);
    const size_t lds = fused_lds_bytes(qmax, sizeof(T));
    // rows of inv(R_ii) are the columns of the stored block transposes, and
    // the reverse for inv(R_ii)^T
    const T *M = trans ? Rinv : Rinv + trinv_elems(n);
    ctqr_status s = fused_setup();
    if (!s) s = fill_u32(bar, GB_WORDS, 0u, st);
    if (s) return s;
    void *args[] = {&n, &S, (void *)&R, (void *)&ldr, (void *)&M, (void *)&C, (void *)&ldc, &X, (void *)&ldx,
                    &E, &bar, (void *)&skip, &info};
    const void *fn = trans ? trsm_fn<T, true>(S) : trsm_fn<T, false>(S);
    HIP_TRY(hipLaunchCooperativeKernel(fn, dim3(G), dim3(FNT), args, lds, st));
    return CTQR_OK;
}

template <typename T>
ctqr_status qtb_fused(int m, int n, int nb, int S, const T *QR, int64_t lda, const T *Tf, const double *B,
                      int64_t ldb, T *Y, int64_t ldy, T *ex, unsigned *bar, ctqr_info *info, hipStream_t st)
{
    if (S < 1 || S > SM || nb < 1 || nb > XCH || nb % CH != 0 || !fused_fits(m, sizeof(T)))
        return CTQR_EUNSUPPORTED;
    const int G = fused_grid();
    const int qmax = (int)ceil_div(ceil_div(m, CH), G);
    const size_t lds = fused_lds_bytes(qmax, sizeof(T));
    T *P = ex, *Wv = P + (size_t)G * nb * SM, *Wt = Wv + (size_t)nb * SM;
    ctqr_status s = fused_setup();
    if (!s) s = fill_u32(bar, GB_WORDS, 0u, st);
    if (s) return s;
    void *args[] = {&m, &n, &nb, &S, (void *)&QR, (void *)&lda, (void *)&Tf, (void *)&B, (void *)&ldb, &Y,
                    (void *)&ldy, &P, &Wv, &Wt, &bar, &info};
    HIP_TRY(hipLaunchCooperativeKernel(qtb_fn<T>(S), dim3(G), dim3(FNT), args, lds, st));
    return CTQR_OK;
}

// exchange elements of the fused kernels: the substitutions' diagonal-block
// vector (TRSM_BIG x FUSED_MAX_S) or Q^T B's partials, W and W' (nb <= 256)
size_t fused_exchange_elems() { return std::max<size_t>((size_t)BIG * SM, ((size_t)fused_grid() + 2) * 256 * SM); }

template ctqr_status trsm_fused<float>(int, int, bool, const float *, int64_t, const float *, const float *, int64_t,
                                       float *, int64_t, float *, unsigned *, const int *, ctqr_info *, hipStream_t);
template ctqr_status trsm_fused<double>(int, int, bool, const double *, int64_t, const double *, const double *,
                                        int64_t, double *, int64_t, double *, unsigned *, const int *, ctqr_info *,
                                        hipStream_t);
template ctqr_status qtb_fused<float>(int, int, int, int, const float *, int64_t, const float *, const double *,
                                      int64_t, float *, int64_t, float *, unsigned *, ctqr_info *, hipStream_t);
template ctqr_status qtb_fused<double>(int, int, int, int, const double *, int64_t, const double *, const double *,
                                       int64_t, double *, int64_t, double *, unsigned *, ctqr_info *, hipStream_t);
