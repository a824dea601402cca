// MFMA GEMMs for the block-reflector applications of the QR path.
//
// Applying a compact-WY block reflector H = I - V T V^T from the left,
// C <- H^T C = C - V (T^T (V^T C)), is the paper's Apply_left_Qt_of_dense_QR
// (Section II-C) and the whole of the trailing update and of Q^T B.  It needs
// two product shapes, both column-major:
//
//   TN:  Out (M x N) = alpha * A^T B + beta * Out,  A: K x M,  B: K x N
//        (W = V^T C and W' = T^T W; the reduction runs down the columns, i.e.
//        along contiguous memory, for both operands; split over K when the
//        output has too few tiles to fill the chip)
//   NN:  C (M x N) += alpha * A B,                  A: M x K,  B: K x N
//        (C -= V W', the rank-nb update, and the block back substitution)
//
// Either operand that is a Householder block V (unit lower trapezoidal: 1 on
// its diagonal, 0 above, the stored vector below) is read straight out of the
// factored matrix with that structure applied while loading, so no separate
// copy of V is kept.
//
// Tiling (gfx950, 64-wide waves): a 256-thread workgroup owns a 128 x 128
// output tile, each of its 4 waves a 64 x 64 sub-tile built from MFMA blocks
// (FP32: v_mfma_f32_32x32x2f32, FP64: v_mfma_f64_16x16x4f64).  Products with
// few output columns (a solve with a handful of slices) use a 128 x 32 tile
// instead, one 32 x 32 sub-tile per wave, so a narrow right-hand side does not
// pay for 128 columns of MFMA work.  The k-step is
// 128 bytes of every operand column (32 floats / 16 doubles), staged through
// double-buffered LDS from 16-byte coalesced global loads.  The MFMA output is
// computed transposed, so that the 32 (FP32) or 16 (FP64) lanes that share an
// output column hold consecutive rows of the column-major result and its
// stores coalesce.  Within a k-group the k index a lane feeds to successive
// MFMAs is permuted (k = 4*slot + s) so each lane fetches 4 consecutive k
// values with one LDS read; the sum over k is unchanged.  Workgroup ids are
// remapped so the tiles one XCD runs are neighbours (shared L2 lines).
//
// BF16 products of FP32 operands, accumulated in FP32.  One part (template
// parameter BF = 1): every operand rounded to bf16, one
// v_mfma_f32_32x32x16_bf16 product.  Split (the *_bf16x3 kernels): each
// operand as a high part h = bf16(x) and a low part l = bf16(x - h), exact to
// about 16 bits, and the three products l h', h l', h h' (the l l' term lies
// below the FP32 accumulation's own rounding for most sums).  The Householder
// block V is split once per block column, in the layout each product reads;
// C, read by only two tiles of [G | W], is split while staged.
#include <cstdint>
#include <cstdlib>
#include <type_traits>

#include "common.h"
#include "kernels.h"

namespace {

constexpr int TILE = 128;     // output tile edge
constexpr int NTHR = 256;     // threads per workgroup
constexpr int GROUP_M = 8;    // row tiles per group in the tile order

template <typename T> struct Mf;
template <> struct Mf<float> {
    static constexpr int BK = 32;      // k per LDS stage (128 bytes)
    static constexpr int MB = 32;      // MFMA block edge
    static constexpr int NBLK = 2;     // MFMA blocks per wave edge (64/MB)
    static constexpr int SLOTS = 2;    // lanes groups sharing a row (64/MB)
    static constexpr int KG = 8;       // k per group of 4 MFMAs
    static constexpr int PAD_KC = 4;   // LDS pad (elements) of [col][k] tiles
    static constexpr int PAD_MK = 8;   // LDS pad (elements) of [k][row] tiles
    using acc_t = floatx16;
};
template <> struct Mf<double> {
    static constexpr int BK = 16;
    static constexpr int MB = 16;
    static constexpr int NBLK = 4;
    static constexpr int SLOTS = 4;
    static constexpr int KG = 16;
    static constexpr int PAD_KC = 2;
    static constexpr int PAD_MK = 4;
    using acc_t = doublex4;
};

__device__ inline floatx16 mfma(float a, float b, floatx16 c)
{
    return __builtin_amdgcn_mfma_f32_32x32x2f32(a, b, c, 0, 0, 0);
}
__device__ inline doublex4 mfma(double a, double b, doublex4 c)
{
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// Maps blockIdx.x to an output tile: XCD-contiguous ranges of logical ids,
// then GROUP_M row tiles sweeping across the column tiles.
__device__ inline void tile_of_block(int tiles_m, int tiles_n, int &tm, int &tn)
{
    int total = tiles_m * tiles_n;
    int id = blockIdx.x;
    int per = total / 8;
    if (id < per * 8) id = (id % 8) * per + id / 8;
    int span = GROUP_M * tiles_n;
    int group = id / span;
    int first = group * GROUP_M;
    int gsize = min(tiles_m - first, GROUP_M);
    int in = id - group * span;
    tm = first + in % gsize;
    tn = in / gsize;
}

// Value of a unit-lower-trapezoidal Householder block at (row, col).
template <typename T>
__device__ inline T vmask(T stored, int row, int col)
{
    return row > col ? stored : (row == col ? T(1) : T(0));
}

// 16-byte vector of E = 16 / sizeof(T) consecutive elements of one column.
template <typename T> struct Vec16;
template <> struct Vec16<float> { using type = floatx4; };
template <> struct Vec16<double> { using type = doublex2; };
template <typename T> using vec16_t = typename Vec16<T>::type;
typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

// Loads are issued unconditionally (an out-of-range chunk reads the operand's
// first chunk instead), so every load of a stage is in flight at once; the
// bounds and the Householder structure are applied when the registers are
// written to LDS, after the MFMA work of the previous stage has hidden the
// load latency.

// ---------------------------------------------------------------------------
// Loader of a COLS-column x BK tile whose columns are contiguous in k
// ("[col][k]" LDS layout, padded), used for both TN operands and for the B
// operand of NN.  Column c of the tile is operand column col0 + c, rows
// k0 .. k0+BK-1.  mask_cols > 0 marks the first mask_cols operand columns as
// a Householder block (diagonal at row == column).
// ---------------------------------------------------------------------------
template <typename T, int COLS = TILE>
struct KcTile {
    static constexpr int BK = Mf<T>::BK;
    static constexpr int LD = BK + Mf<T>::PAD_KC;
    static constexpr int E = 16 / sizeof(T);
    static constexpr int CPC = BK / E;                 // chunks per column (8)
    static constexpr int PER_THR = COLS * CPC / NTHR;  // 4 (1 for a 32-column tile)
    static_assert(COLS * CPC % NTHR == 0, "tile does not split evenly over the workgroup");
    vec16_t<T> r[PER_THR];
    int col0_, k0_, kmax_, ncols_, mask_;

    __device__ inline void load(const T *P, int64_t ld, int ncols, int col0, int k0, int kmax,
                                int mask_cols)
    {
        col0_ = col0; k0_ = k0; kmax_ = kmax; ncols_ = ncols; mask_ = mask_cols;
#pragma unroll
        for (int q = 0; q < PER_THR; ++q) {
            int f = threadIdx.x + NTHR * q;
            int c = f / CPC, h = f % CPC;
            int col = col0 + c, k = k0 + h * E;
            bool ok = col < ncols && k < kmax;
            const T *p = ok ? P + (int64_t)col * ld + k : P;
            r[q] = *reinterpret_cast<const vec16_t<T> *>(p);
        }
    }
    // register chunk q with the bounds and the Householder structure applied;
    // c, h: its column and chunk within the tile
    __device__ inline vec16_t<T> masked(int q, int &c, int &h) const
    {
        int f = threadIdx.x + NTHR * q;
        c = f / CPC;
        h = f % CPC;
        int col = col0_ + c, k = k0_ + h * E;
        vec16_t<T> v = r[q];
        if (col >= ncols_ || k + E > kmax_ || (col < mask_ && k <= col)) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                T x = (col < ncols_ && k + e < kmax_) ? v[e] : T(0);
                v[e] = col < mask_ ? vmask(x, k + e, col) : x;
            }
        }
        return v;
    }
    __device__ inline void store(T *lds) const
    {
#pragma unroll
        for (int q = 0; q < PER_THR; ++q) {
            int c, h;
            vec16_t<T> v = masked(q, c, h);
            *reinterpret_cast<vec16_t<T> *>(lds + c * LD + h * E) = v;
        }
    }
    // BF16 staging (FP32 operands): the same values rounded to bf16 (nearest
    // even), [col][k] layout with row stride LDB
    static constexpr int LDB = BK + 8;
    __device__ inline void store_bf(__bf16 *lds) const
    {
        static_assert(sizeof(T) == 4, "bf16 staging of FP32 operands only");
#pragma unroll
        for (int q = 0; q < PER_THR; ++q) {
            int c, h;
            vec16_t<T> v = masked(q, c, h);
            bf16x4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = (__bf16)v[e];
            *reinterpret_cast<bf16x4 *>(lds + c * LDB + h * E) = o;
        }
    }
    // split staging: high parts to hi, the bf16-rounded remainders to lo
    __device__ inline void store_bf2(__bf16 *hi, __bf16 *lo) const
    {
        static_assert(sizeof(T) == 4, "bf16 staging of FP32 operands only");
#pragma unroll
        for (int q = 0; q < PER_THR; ++q) {
            int c, h;
            vec16_t<T> v = masked(q, c, h);
            bf16x4 oh, ol;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const __bf16 t = (__bf16)v[e];
                oh[e] = t;
                ol[e] = (__bf16)(v[e] - (float)t);
            }
            *reinterpret_cast<bf16x4 *>(hi + c * LDB + h * E) = oh;
            *reinterpret_cast<bf16x4 *>(lo + c * LDB + h * E) = ol;
        }
    }
};

// Loader of a BK-column x 128-row tile of a column-major M x K operand
// ("[k][row]" LDS layout), the A operand of NN.  mask: operand is a
// Householder block (value at (row, k) is 1 on row == k, 0 above).
template <typename T>
struct MkTile {
    static constexpr int BK = Mf<T>::BK;
    static constexpr int LD = TILE + Mf<T>::PAD_MK;
    static constexpr int E = 16 / sizeof(T);
    static constexpr int CPC = TILE / E;                // chunks per column (32/64)
    static constexpr int PER_THR = BK * CPC / NTHR;     // 4
    vec16_t<T> r[PER_THR];
    int row0_, k0_, kmax_, mrows_;
    bool mask_;

    __device__ inline void load(const T *P, int64_t ld, int mrows, int row0, int k0, int kmax,
                                bool mask)
    {
        row0_ = row0; k0_ = k0; kmax_ = kmax; mrows_ = mrows; mask_ = mask;
#pragma unroll
        for (int q = 0; q < PER_THR; ++q) {
            int f = threadIdx.x + NTHR * q;
            int kk = f / CPC, h = f % CPC;
            int k = k0 + kk, row = row0 + h * E;
            bool ok = k < kmax && row < mrows;
            const T *p = ok ? P + (int64_t)k * ld + row : P;
            r[q] = *reinterpret_cast<const vec16_t<T> *>(p);
        }
    }
    __device__ inline vec16_t<T> masked(int q, int &kk, int &h) const
    {
        int f = threadIdx.x + NTHR * q;
        kk = f / CPC;
        h = f % CPC;
        int k = k0_ + kk, row = row0_ + h * E;
        vec16_t<T> v = r[q];
        if (k >= kmax_ || row + E > mrows_ || (mask_ && row <= k)) {
#pragma unroll
            for (int e = 0; e < E; ++e) {
                T x = (k < kmax_ && row + e < mrows_) ? v[e] : T(0);
                v[e] = mask_ ? vmask(x, row + e, k) : x;
            }
        }
        return v;
    }
    __device__ inline void store(T *lds) const
    {
#pragma unroll
        for (int q = 0; q < PER_THR; ++q) {
            int kk, h;
            vec16_t<T> v = masked(q, kk, h);
            *reinterpret_cast<vec16_t<T> *>(lds + kk * LD + h * E) = v;
        }
    }
};

// BF16 loader of the same BK-column x 128-row tile (FP32, column-major
// M x K): each thread takes one row and four groups of 4 consecutive k, so
// it can write the row's bf16 values for those k as one 8-byte LDS store in
// the [row][k] layout the BF16 MFMA reads.  The global loads are single
// floats, still coalesced: the 64 lanes of a wave read 64 consecutive rows of
// one column.
template <typename T>
struct MkTileBf {
    static_assert(sizeof(T) == 4, "bf16 staging of FP32 operands only");
    static constexpr int BK = Mf<T>::BK;
    static constexpr int LDB = BK + 8;
    static constexpr int QUADS = BK / 4;                   // k groups per row (8)
    static constexpr int PER_THR = TILE * QUADS / NTHR;    // groups per thread (4)
    static constexpr int QSTEP = NTHR / TILE;              // 2
    T r[PER_THR][4];
    int row0_, k0_, kmax_, mrows_;
    bool mask_;

    __device__ inline void load(const T *P, int64_t ld, int mrows, int row0, int k0, int kmax, bool mask)
    {
        row0_ = row0; k0_ = k0; kmax_ = kmax; mrows_ = mrows; mask_ = mask;
        const int row = row0 + (int)threadIdx.x % TILE;
#pragma unroll
        for (int j = 0; j < PER_THR; ++j) {
            const int q = (int)threadIdx.x / TILE + QSTEP * j;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const int k = k0 + 4 * q + e;
                const bool ok = k < kmax && row < mrows;
                r[j][e] = *(ok ? P + (int64_t)k * ld + row : P);
            }
        }
    }
    // the 4 values of group j with the bounds and the Householder structure
    __device__ inline void masked(int j, int &rr, int &q, T (&v)[4]) const
    {
        rr = (int)threadIdx.x % TILE;
        q = (int)threadIdx.x / TILE + QSTEP * j;
        const int row = row0_ + rr;
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const int k = k0_ + 4 * q + e;
            const T x = (k < kmax_ && row < mrows_) ? r[j][e] : T(0);
            v[e] = mask_ ? vmask(x, row, k) : x;
        }
    }
    __device__ inline void store_bf(__bf16 *lds) const
    {
#pragma unroll
        for (int j = 0; j < PER_THR; ++j) {
            int rr, q;
            T v[4];
            masked(j, rr, q, v);
            bf16x4 o;
#pragma unroll
            for (int e = 0; e < 4; ++e) o[e] = (__bf16)v[e];
            *reinterpret_cast<bf16x4 *>(lds + rr * LDB + 4 * q) = o;
        }
    }
};

// One BK-deep step of a wave's (NI*MB) x (NJ*MB) MFMA accumulation from LDS.
// opA: [n][k] tile (MFMA rows = output columns n), opB: [m][k] tile when
// B_KC (TN) or [k][m] tile otherwise (NN).  Output block (ib, jb) covers
// output columns wn + ib*MB .. and rows wm + jb*MB ..
template <typename T, bool B_KC, int NI, int NJ>
__device__ inline void mfma_step(const T *opA, const T *opB, int wn, int wm,
                                 typename Mf<T>::acc_t (&acc)[NI][NJ])
{
    using M = Mf<T>;
    const int lane = threadIdx.x % CTQR_WAVE;
    const int li = lane % M::MB, slot = lane / M::MB;
    if constexpr (sizeof(T) == 8) {
        // FP64: 4x4 blocks; fetch two k values per operand at a time to keep
        // the register footprint inside two waves per SIMD.
        const int kk = 4 * slot;
#pragma unroll
        for (int sp = 0; sp < 2; ++sp) {
            doublex2 a[NI], b[NJ];
#pragma unroll
            for (int ib = 0; ib < NI; ++ib)
                a[ib] = *reinterpret_cast<const doublex2 *>(opA + (wn + ib * M::MB + li) * KcTile<T>::LD + kk + 2 * sp);
#pragma unroll
            for (int jb = 0; jb < NJ; ++jb) {
                if constexpr (B_KC) {
                    b[jb] = *reinterpret_cast<const doublex2 *>(opB + (wm + jb * M::MB + li) * KcTile<T>::LD + kk + 2 * sp);
                } else {
                    const T *p = opB + (kk + 2 * sp) * MkTile<T>::LD + wm + jb * M::MB + li;
                    b[jb][0] = p[0];
                    b[jb][1] = p[MkTile<T>::LD];
                }
            }
#pragma unroll
            for (int s = 0; s < 2; ++s)
#pragma unroll
                for (int ib = 0; ib < NI; ++ib)
#pragma unroll
                    for (int jb = 0; jb < NJ; ++jb)
                        acc[ib][jb] = mfma(a[ib][s], b[jb][s], acc[ib][jb]);
        }
        return;
    }
    // FP32: 4 k-groups of 8 per stage; the LDS fragments of k-group g+1 are
    // fetched into the second register set while the 16 MFMAs of group g issue.
    constexpr int NG = M::BK / M::KG;
    floatx4 a[2][NI], b[2][NJ];
    auto fetch = [&](int g, int buf) {
        const int kk = g * M::KG + 4 * slot;
#pragma unroll
        for (int ib = 0; ib < NI; ++ib)
            a[buf][ib] = *reinterpret_cast<const floatx4 *>(opA + (wn + ib * M::MB + li) * KcTile<T>::LD + kk);
#pragma unroll
        for (int jb = 0; jb < NJ; ++jb) {
            if constexpr (B_KC) {
                b[buf][jb] = *reinterpret_cast<const floatx4 *>(opB + (wm + jb * M::MB + li) * KcTile<T>::LD + kk);
            } else {
                const T *p = opB + kk * MkTile<T>::LD + wm + jb * M::MB + li;
#pragma unroll
                for (int s = 0; s < 4; ++s) b[buf][jb][s] = p[s * MkTile<T>::LD];
            }
        }
    };
    fetch(0, 0);
#pragma unroll
    for (int g = 0; g < NG; ++g) {
        const int cb = g & 1;
        if (g + 1 < NG) fetch(g + 1, cb ^ 1);
#pragma unroll
        for (int s = 0; s < 4; ++s)
#pragma unroll
            for (int ib = 0; ib < NI; ++ib)
#pragma unroll
                for (int jb = 0; jb < NJ; ++jb)
                    acc[ib][jb] = mfma(a[cb][ib][s], b[cb][jb][s], acc[ib][jb]);
    }
}

// One BK-deep step of a wave's MFMA accumulation from bf16 LDS tiles (both
// [col][k], row stride LDB): v_mfma_f32_32x32x16_bf16, FP32 accumulation.
// Each lane feeds 8 consecutive k of its row (k = 16 g + 8 slot + e) to both
// operands, so the sum covers every k once.
template <int NI, int NJ>
__device__ inline void mfma_step_bf(const __bf16 *opA, const __bf16 *opB, int wn, int wm,
                                    floatx16 (&acc)[NI][NJ])
{
    constexpr int LDB = KcTile<float>::LDB;
    const int lane = threadIdx.x % CTQR_WAVE;
    const int li = lane % 32, slot = lane / 32;
#pragma unroll
    for (int g = 0; g < Mf<float>::BK / 16; ++g) {
        const int kk = 16 * g + 8 * slot;
        bf16x8 a[NI], b[NJ];
#pragma unroll
        for (int ib = 0; ib < NI; ++ib)
            a[ib] = *reinterpret_cast<const bf16x8 *>(opA + (wn + ib * 32 + li) * LDB + kk);
#pragma unroll
        for (int jb = 0; jb < NJ; ++jb)
            b[jb] = *reinterpret_cast<const bf16x8 *>(opB + (wm + jb * 32 + li) * LDB + kk);
#pragma unroll
        for (int ib = 0; ib < NI; ++ib)
#pragma unroll
            for (int jb = 0; jb < NJ; ++jb)
                acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[ib], b[jb], acc[ib][jb], 0, 0, 0);
    }
}

// The same step from split operands (high and low bf16 parts, same layout):
// per block the low-part products first, then the high-high product.  Each
// of the three products is issued for every block before the next product,
// so consecutive MFMAs never wait on each other's accumulator; every block
// still takes its three products in that order.
template <int NI, int NJ>
__device__ inline void mfma_step_bf2(const __bf16 *opAh, const __bf16 *opAl, const __bf16 *opBh,
                                     const __bf16 *opBl, int wn, int wm, floatx16 (&acc)[NI][NJ])
{
    constexpr int LDB = KcTile<float>::LDB;
    const int lane = threadIdx.x % CTQR_WAVE;
    const int li = lane % 32, slot = lane / 32;
#pragma unroll
    for (int g = 0; g < Mf<float>::BK / 16; ++g) {
        const int kk = 16 * g + 8 * slot;
        bf16x8 bh[NJ], bl[NJ], ah[NI], al[NI];
#pragma unroll
        for (int jb = 0; jb < NJ; ++jb) {
            bh[jb] = *reinterpret_cast<const bf16x8 *>(opBh + (wm + jb * 32 + li) * LDB + kk);
            bl[jb] = *reinterpret_cast<const bf16x8 *>(opBl + (wm + jb * 32 + li) * LDB + kk);
        }
#pragma unroll
        for (int ib = 0; ib < NI; ++ib) {
            ah[ib] = *reinterpret_cast<const bf16x8 *>(opAh + (wn + ib * 32 + li) * LDB + kk);
            al[ib] = *reinterpret_cast<const bf16x8 *>(opAl + (wn + ib * 32 + li) * LDB + kk);
        }
#pragma unroll
        for (int ib = 0; ib < NI; ++ib)
#pragma unroll
            for (int jb = 0; jb < NJ; ++jb)
                acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[ib], bh[jb], acc[ib][jb], 0, 0, 0);
#pragma unroll
        for (int ib = 0; ib < NI; ++ib)
#pragma unroll
            for (int jb = 0; jb < NJ; ++jb)
                acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ib], bl[jb], acc[ib][jb], 0, 0, 0);
#pragma unroll
        for (int ib = 0; ib < NI; ++ib)
#pragma unroll
            for (int jb = 0; jb < NJ; ++jb)
                acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ib], bh[jb], acc[ib][jb], 0, 0, 0);
    }
}

// Bank-conflict-free LDS layout of the 8-wave update: rows of 32 bf16 (64 B,
// no padding), the 16-byte chunk c of row r stored at chunk c ^ ((r / 4) % 4).
// The 16 rows a quarter wave reads (or the 4 rows x 4 chunks it writes) then
// fall on 16 distinct 16-byte bank groups of the 64-bank LDS.
__device__ inline int swz_off(int r, int c) { return r * 32 + 8 * (c ^ ((r >> 2) & 3)); }

// mfma_step_bf2 on that layout (the same products in the same order)
template <int NI, int NJ>
__device__ inline void mfma_step_bf2_swz(const __bf16 *opAh, const __bf16 *opAl, const __bf16 *opBh,
                                         const __bf16 *opBl, int wn, int wm, floatx16 (&acc)[NI][NJ])
{
    const int lane = threadIdx.x % CTQR_WAVE;
    const int li = lane % 32, slot = lane / 32;
#pragma unroll
    for (int g = 0; g < Mf<float>::BK / 16; ++g) {
        const int c = 2 * g + slot;
        bf16x8 bh[NJ], bl[NJ], ah[NI], al[NI];
#pragma unroll
        for (int jb = 0; jb < NJ; ++jb) {
            bh[jb] = *reinterpret_cast<const bf16x8 *>(opBh + swz_off(wm + jb * 32 + li, c));
            bl[jb] = *reinterpret_cast<const bf16x8 *>(opBl + swz_off(wm + jb * 32 + li, c));
        }
#pragma unroll
        for (int ib = 0; ib < NI; ++ib) {
            ah[ib] = *reinterpret_cast<const bf16x8 *>(opAh + swz_off(wn + ib * 32 + li, c));
            al[ib] = *reinterpret_cast<const bf16x8 *>(opAl + swz_off(wn + ib * 32 + li, c));
        }
#pragma unroll
        for (int ib = 0; ib < NI; ++ib)
#pragma unroll
            for (int jb = 0; jb < NJ; ++jb)
                acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(al[ib], bh[jb], acc[ib][jb], 0, 0, 0);
#pragma unroll
        for (int ib = 0; ib < NI; ++ib)
#pragma unroll
            for (int jb = 0; jb < NJ; ++jb)
                acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ib], bl[jb], acc[ib][jb], 0, 0, 0);
#pragma unroll
        for (int ib = 0; ib < NI; ++ib)
#pragma unroll
            for (int jb = 0; jb < NJ; ++jb)
                acc[ib][jb] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(ah[ib], bh[jb], acc[ib][jb], 0, 0, 0);
    }
}

// Output coordinates of accumulator element r of block (ib, jb) for this lane:
// output column (n) and row (m) offsets inside the wave's 64x64 sub-tile.
template <typename T>
__device__ inline void acc_coords(int ib, int jb, int r, int &n, int &m)
{
    using M = Mf<T>;
    const int lane = threadIdx.x % CTQR_WAVE;
    if constexpr (sizeof(T) == 4) {
        n = ib * 32 + 8 * (r / 4) + 4 * (lane / 32) + (r % 4);
        m = jb * 32 + lane % 32;
    } else {
        // v_mfma_f64_16x16x4f64: register r of lane l holds row 4r + l/16
        n = ib * 16 + 4 * r + lane / 16;
        m = jb * 16 + lane % 16;
    }
    (void)sizeof(M);
}

template <typename T> constexpr int acc_len() { return sizeof(T) == 4 ? 16 : 4; }

// Wave layout of a 128 x TW output tile (TW = 128 or 32 output columns): each
// wave owns an EDGE x EDGE sub-tile of NI x NJ MFMA blocks at (wn, wm).
template <typename T, int TW>
struct WaveTile {
    static_assert(TW == TILE || TW == 32, "output tile width is 128 or 32");
    static constexpr int EDGE = TW == TILE ? 64 : 32;
    static constexpr int NI = EDGE / Mf<T>::MB;   // blocks along output columns
    static constexpr int NJ = EDGE / Mf<T>::MB;   // blocks along output rows
    __device__ static inline int wn(int wave) { return TW == TILE ? (wave / 2) * 64 : 0; }
    __device__ static inline int wm(int wave) { return TW == TILE ? (wave % 2) * 64 : wave * 32; }
};

// ---------------------------------------------------------------------------
// TN:  Out = alpha * A^T B + beta * Out   (or split-K partials)
// ---------------------------------------------------------------------------
// TP: the output is written transposed (element (m, n) of Out at m ldo + n,
// of split z's partial at (z M + m) N + n): a product formed as B^T A on the
// narrow tile lands where A^T B would.
template <typename T, int TW, int BF, bool TP = false>
__global__ __launch_bounds__(NTHR, 2)
void gemm_tn_kernel(int M, int N, int K,
                    const T *__restrict__ A, int64_t lda, int amask,
                    const T *__restrict__ B, int64_t ldb, int bmask,
                    T alpha, T beta, T *__restrict__ Out, int64_t ldo,
                    T *__restrict__ part, int kchunk, const int *skip, int tri)
{
    using Mt = Mf<T>;
    using W = WaveTile<T, TW>;
    if (skip && *skip) return;
    // BF = 1: FP32 operands rounded to bf16 while staged (BF16 MFMA, FP32
    // accumulation; split operands: gemm_tn_bf16x3_kernel)
    static_assert(BF == 0 || (sizeof(T) == 4 && TW == TILE && BF == 1), "bf16 path: FP32, 128-wide tiles");
    using LT = typename std::conditional<(BF > 0), __bf16, T>::type;
    constexpr int LDX = BF ? KcTile<T>::LDB : KcTile<T>::LD;
    __shared__ __attribute__((aligned(16))) LT sA[2][TILE * LDX];
    __shared__ __attribute__((aligned(16))) LT sB[2][TW * LDX];

    int tm, tn;
    tile_of_block((M + TILE - 1) / TILE, (N + TW - 1) / TW, tm, tn);
    const int m0 = tm * TILE, n0 = tn * TW;
    // tri: A(k, m) is zero for k < m (1) or for k > m (2), so the tile's rows
    // need only k >= m0, or k < m0 + TILE (whole BK steps of exact zeros
    // skipped: the same sums)
    const int kbeg = tri == 1 ? max((int)blockIdx.z * kchunk, m0) : (int)blockIdx.z * kchunk;
    const int kend = tri == 2 ? min(min(K, (int)blockIdx.z * kchunk + kchunk), m0 + TILE)
                              : min(K, (int)blockIdx.z * kchunk + kchunk);
    const int wave = threadIdx.x / CTQR_WAVE;
    const int wn = W::wn(wave), wm = W::wm(wave);

    typename Mt::acc_t acc[W::NI][W::NJ];
#pragma unroll
    for (int i = 0; i < W::NI; ++i)
#pragma unroll
        for (int j = 0; j < W::NJ; ++j)
#pragma unroll
            for (int e = 0; e < acc_len<T>(); ++e) acc[i][j][e] = T(0);

    KcTile<T> la;
    KcTile<T, TW> lb;
    auto stage = [](const KcTile<T> &a, const KcTile<T, TW> &b, LT *da, LT *db) {
        if constexpr (BF == 1) {
            a.store_bf(da);
            b.store_bf(db);
        } else {
            a.store(da);
            b.store(db);
        }
    };
    if (kbeg < kend) {
        la.load(A, lda, M, m0, kbeg, kend, amask);
        lb.load(B, ldb, N, n0, kbeg, kend, bmask);
        stage(la, lb, sA[0], sB[0]);
    }
    __syncthreads();
    int cur = 0;
    for (int k = kbeg; k < kend; k += Mt::BK) {
        const bool more = k + Mt::BK < kend;
        if (more) {
            la.load(A, lda, M, m0, k + Mt::BK, kend, amask);
            lb.load(B, ldb, N, n0, k + Mt::BK, kend, bmask);
        }
        if constexpr (BF == 1)
            mfma_step_bf<W::NI, W::NJ>(sB[cur], sA[cur], wn, wm, acc);
        else
            mfma_step<T, true, W::NI, W::NJ>(sB[cur], sA[cur], wn, wm, acc);
        if (more) stage(la, lb, sA[cur ^ 1], sB[cur ^ 1]);
        __syncthreads();
        cur ^= 1;
    }

    const bool split = gridDim.z > 1;
#pragma unroll
    for (int ib = 0; ib < W::NI; ++ib)
#pragma unroll
        for (int jb = 0; jb < W::NJ; ++jb)
#pragma unroll
            for (int r = 0; r < acc_len<T>(); ++r) {
                int n, m;
                acc_coords<T>(ib, jb, r, n, m);
                n += n0 + wn;
                m += m0 + wm;
                if (m < M && n < N) {
                    T v = acc[ib][jb][r];
                    if (split) {
                        part[TP ? ((int64_t)blockIdx.z * M + m) * N + n : ((int64_t)blockIdx.z * N + n) * M + m] = v;
                    } else {
                        T *o = TP ? Out + (int64_t)m * ldo + n : Out + (int64_t)n * ldo + m;
                        *o = beta == T(0) ? alpha * v : alpha * v + beta * *o;
                    }
                }
            }
}

// Deterministic split-K reduction: Out = alpha * sum_z part[z] + beta * Out.
// A workgroup of SG waves owns 64 consecutive outputs: wave w sums the
// partials of splits w, w + SG, w + 2 SG, ... in order, then the SG wave sums
// are added in wave order.
template <typename T, int SG>
__global__ __launch_bounds__(64 * SG)
void splitk_reduce_kernel(int M, int N, int splits, const T *__restrict__ part,
                          T alpha, T beta, T *__restrict__ Out, int64_t ldo,
                          const int *skip)
{
    if (skip && *skip) return;
    __shared__ T red[SG][64];
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    const int64_t idx = (int64_t)blockIdx.x * 64 + lane;
    const int64_t total = (int64_t)M * N;
    T acc = T(0);
    if (idx < total) {
#pragma unroll 4
        for (int z = w; z < splits; z += SG) acc += part[(int64_t)z * total + idx];
    }
    red[w][lane] = acc;
    __syncthreads();
    if (w == 0 && idx < total) {
        T v = red[0][lane];
#pragma unroll
        for (int k = 1; k < SG; ++k) v += red[k][lane];
        const int n = (int)(idx / M), m = (int)(idx % M);
        T *o = Out + (int64_t)n * ldo + m;
        *o = beta == T(0) ? alpha * v : alpha * v + beta * *o;
    }
}

// W2 = Tt^T W for W = the sum of `splits` partials of an M x N product (M <=
// 32; partial z of element (m, n) at src[z zstride + n ld + m]), one
// workgroup of 16 waves per two columns: the sum in the order of
// splitk_reduce_kernel<T, 16>, then each output as sum_k Tt(k, m) W(k, n) in
// k order.
template <typename T>
__global__ __launch_bounds__(1024)
void tprod_reduce_kernel(int M, int N, int splits, const T *__restrict__ src, int64_t ld, int64_t zstride,
                         const T *__restrict__ Tt, int64_t ldt, T *__restrict__ W2, int64_t ldw)
{
    __shared__ T red[16][64];
    __shared__ T col[64];
    const int lane = threadIdx.x % 64, w = threadIdx.x / 64;
    const int c = lane / 32, m = lane % 32;
    const int n = blockIdx.x * 2 + c;
    const bool ok = n < N && m < M;
    T acc = T(0);
    if (ok) {
#pragma unroll 4
        for (int z = w; z < splits; z += 16) acc += src[(int64_t)z * zstride + (int64_t)n * ld + m];
    }
    red[w][lane] = acc;
    __syncthreads();
    if (w == 0) {
        T v = red[0][lane];
#pragma unroll
        for (int k = 1; k < 16; ++k) v += red[k][lane];
        col[lane] = ok ? v : T(0);
    }
    __syncthreads();
    if (w == 0 && ok) {
        T s = T(0);
        for (int k = 0; k < M; ++k) s += Tt[(int64_t)m * ldt + k] * col[32 * c + k];
        W2[(int64_t)n * ldw + m] = s;
    }
}

// ---------------------------------------------------------------------------
// NN:  C += alpha * A B   (A: M x K, optionally a Householder block; B: K x N)
// ---------------------------------------------------------------------------
// KIND only separates the symbols of the launch sites in a profile: 1 is the
// trailing update of the factorization, 0 every other use.
template <typename T, int KIND, int TW, bool SPLIT, int BF>
__global__ __launch_bounds__(NTHR, 2)
void gemm_nn_kernel(int M, int N, int K,
                    const T *__restrict__ A, int64_t lda, int amask,
                    const T *__restrict__ B, int64_t ldb,
                    T alpha, T *__restrict__ C, int64_t ldc, int accum,
                    T *__restrict__ part, int kchunk, const int *skip, int64_t bsa, int64_t bsb, int64_t bsc)
{
    // accum != 0: C += alpha A B;  accum == 0: C = alpha A B (C is not read).
    // blockIdx.y: product of a batch whose operands lie bsa, bsb, bsc apart.
    // SPLIT: split blockIdx.z covers k in [z kchunk, (z+1) kchunk) and writes
    // its raw product to part (reduced by splitk_reduce_kernel).  A
    // compile-time switch: the unsplit kernels carry none of its registers.
    using Mt = Mf<T>;
    using W = WaveTile<T, TW>;
    if (skip && *skip) return;
    A += (int64_t)blockIdx.y * bsa;
    B += (int64_t)blockIdx.y * bsb;
    C += (int64_t)blockIdx.y * bsc;
    // BF > 0: FP32 operands staged as BF bf16 parts (BF16 MFMA, FP32
    // accumulation); the A tile is then stored [row][k]
    static_assert(BF == 0 || (sizeof(T) == 4 && TW == TILE && !SPLIT && BF == 1),
                  "bf16 path: FP32, 128-wide, unsplit, one part (split parts: gemm_nn_bf16x3_kernel)");
    using LT = typename std::conditional<(BF > 0), __bf16, T>::type;
    constexpr int SA = BF ? TILE * (Mt::BK + 8) : Mt::BK * MkTile<T>::LD;
    constexpr int SB = TW * (BF ? KcTile<T>::LDB : KcTile<T>::LD);
    __shared__ __attribute__((aligned(16))) LT sA[2][SA];
    __shared__ __attribute__((aligned(16))) LT sB[2][SB];

    int tm, tn;
    tile_of_block((M + TILE - 1) / TILE, (N + TW - 1) / TW, tm, tn);
    const int m0 = tm * TILE, n0 = tn * TW;
    const int wave = threadIdx.x / CTQR_WAVE;
    const int wn = W::wn(wave), wm = W::wm(wave);

    typename Mt::acc_t acc[W::NI][W::NJ];
#pragma unroll
    for (int i = 0; i < W::NI; ++i)
#pragma unroll
        for (int j = 0; j < W::NJ; ++j)
#pragma unroll
            for (int e = 0; e < acc_len<T>(); ++e) acc[i][j][e] = T(0);

    constexpr bool split = SPLIT;
    const int kbeg = SPLIT ? (int)blockIdx.z * kchunk : 0;
    const int kend = SPLIT ? min(K, kbeg + kchunk) : K;
    if (SPLIT) accum = 0;
    (void)part;
    (void)kchunk;

    // FP32: fetch the C tile now; its HBM latency hides behind the K loop
    constexpr bool PRE = sizeof(T) == 4;
    T cpre[PRE ? W::NI : 1][PRE ? W::NJ : 1][PRE ? 16 : 1];
    if constexpr (PRE) {
#pragma unroll
        for (int ib = 0; ib < W::NI; ++ib)
#pragma unroll
            for (int jb = 0; jb < W::NJ; ++jb)
#pragma unroll
                for (int r = 0; r < 16; ++r) {
                    int n, m;
                    acc_coords<T>(ib, jb, r, n, m);
                    n += n0 + wn;
                    m += m0 + wm;
                    cpre[ib][jb][r] = (accum && m < M && n < N) ? C[(int64_t)n * ldc + m] : T(0);
                }
    }

    using ATile = typename std::conditional<(BF > 0), MkTileBf<T>, MkTile<T>>::type;
    ATile la;
    KcTile<T, TW> lb;
    auto stage = [](const ATile &a, const KcTile<T, TW> &b, LT *da, LT *db) {
        if constexpr (BF == 1) {
            a.store_bf(da);
            b.store_bf(db);
        } else {
            a.store(da);
            b.store(db);
        }
    };
    la.load(A, lda, M, m0, kbeg, kend, amask != 0);
    lb.load(B, ldb, N, n0, kbeg, kend, 0);
    stage(la, lb, sA[0], sB[0]);
    __syncthreads();
    int cur = 0;
    for (int k = kbeg; k < kend; k += Mt::BK) {
        const bool more = k + Mt::BK < kend;
        if (more) {
            la.load(A, lda, M, m0, k + Mt::BK, kend, amask != 0);
            lb.load(B, ldb, N, n0, k + Mt::BK, kend, 0);
        }
        if constexpr (BF == 1)
            mfma_step_bf<W::NI, W::NJ>(sB[cur], sA[cur], wn, wm, acc);
        else
            mfma_step<T, false, W::NI, W::NJ>(sB[cur], sA[cur], wn, wm, acc);
        if (more) stage(la, lb, sA[cur ^ 1], sB[cur ^ 1]);
        __syncthreads();
        cur ^= 1;
    }

#pragma unroll
    for (int ib = 0; ib < W::NI; ++ib)
#pragma unroll
        for (int jb = 0; jb < W::NJ; ++jb)
#pragma unroll
            for (int r = 0; r < acc_len<T>(); ++r) {
                int n, m;
                acc_coords<T>(ib, jb, r, n, m);
                n += n0 + wn;
                m += m0 + wm;
                if (m < M && n < N) {
                    if constexpr (split) {
                        part[((int64_t)blockIdx.z * N + n) * M + m] = acc[ib][jb][r];
                        continue;
                    }
                    T *c = C + (int64_t)n * ldc + m;
                    if constexpr (PRE)
                        *c = cpre[ib][jb][r] + alpha * acc[ib][jb][r];
                    else
                        *c = accum ? *c + alpha * acc[ib][jb][r] : alpha * acc[ib][jb][r];
                }
            }
}

// ---------------------------------------------------------------------------
// Split-BF16 trailing update from operands split once per block column
// ---------------------------------------------------------------------------
// C -= V W' re-stages every V tile for each column tile and every W' tile for
// each row tile.  Splitting both once into high and low bf16 parts -- V into
// a [row][k] layout, W' in its own [col][k] layout, both zero-padded to whole
// tiles and k stages -- leaves the product kernel no conversion and no
// masking: a stage is four 16-byte copies per thread into LDS.

// V (rows x kc Householder block: unit lower trapezoidal, column-major) to
// high / low bf16 parts, row-major with row stride ldv (k contiguous); rows up
// to rows_pad and k up to ldv are zero.  A workgroup transposes a 64-row x
// 64-k tile through LDS: the 64 lanes of a wave read 64 consecutive rows of a
// column, then eight lanes write one row's 64 k (128 bytes) of each part.
constexpr int SPLIT_V_T = 64;
__global__ __launch_bounds__(256)
void split_v_kernel(int rows, int kc, const float *__restrict__ V, int64_t lda, int rows_pad, int ldv,
                    __bf16 *__restrict__ hi, __bf16 *__restrict__ lo, int mask, const int *skip)
{
    if (skip && *skip) return;
    __shared__ float tile[SPLIT_V_T][SPLIT_V_T + 1];   // [k][row]
    const int r0 = (int)blockIdx.x * SPLIT_V_T, k0 = (int)blockIdx.y * SPLIT_V_T;
    const int t = (int)threadIdx.x;
    {
        const int r = r0 + t % 64, kq = t / 64;
#pragma unroll
        for (int e = 0; e < 16; ++e) {
            const int kl = 16 * kq + e, k = k0 + kl;
            float x = 0.0f;
            if (r < rows && k < kc) {
                const float a = V[(int64_t)k * lda + r];
                x = mask ? vmask(a, r, k) : a;
            }
            tile[kl][t % 64] = x;
        }
    }
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 2; ++q) {
        const int f = t + 256 * q, rl = f / 8, c = f % 8;
        const int r = r0 + rl, k = k0 + 8 * c;
        if (r >= rows_pad || k >= ldv) continue;
        bf16x8 oh, ol;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            const float x = tile[8 * c + e][rl];
            const __bf16 h = (__bf16)x;
            oh[e] = h;
            ol[e] = (__bf16)(x - (float)h);
        }
        *reinterpret_cast<bf16x8 *>(hi + (int64_t)r * ldv + k) = oh;
        *reinterpret_cast<bf16x8 *>(lo + (int64_t)r * ldv + k) = ol;
    }
}

// W' (kc x cols, column-major, leading dimension ldw_in) to high / low bf16
// parts with leading dimension ldw; columns up to cols_pad and k up to ldw are
// zero.  Thread: one column, 8 consecutive k.
__global__ __launch_bounds__(256)
void split_w_kernel(int kc, int cols, const float *__restrict__ W, int64_t ldw_in, int cols_pad, int ldw,
                    __bf16 *__restrict__ hi, __bf16 *__restrict__ lo, const int *skip)
{
    if (skip && *skip) return;
    const int groups = ldw / 8;
    const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (f >= (int64_t)cols_pad * groups) return;
    const int c = (int)(f / groups), k0 = 8 * (int)(f % groups);
    bf16x8 oh, ol;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int k = k0 + e;
        const float x = (c < cols && k < kc) ? W[(int64_t)c * ldw_in + k] : 0.0f;
        const __bf16 t = (__bf16)x;
        oh[e] = t;
        ol[e] = (__bf16)(x - (float)t);
    }
    *reinterpret_cast<bf16x8 *>(hi + (int64_t)c * ldw + k0) = oh;
    *reinterpret_cast<bf16x8 *>(lo + (int64_t)c * ldw + k0) = ol;
}

// C += alpha V W' from the split parts: 128 x 128 output tiles, three BF16
// products per operand pair (mfma_step_bf2), FP32 accumulation, C prefetched
// at the start as in the FP32 trailing update.  C is read and written once,
// with non-temporal accesses, so the streaming tiles do not push the operand
// panels that neighbouring tiles re-read out of the L2.  Ah/Al: rows padded to
// whole tiles, row stride lda; Bh/Bl: columns padded to whole tiles, column
// stride ldb; both cover k up to K rounded up to a stage.  KIND only separates
// the launch sites in a profile: 1 is the factorization's trailing update (the
// launches too small for the 8-wave form), 2 the update of the rest of a group
// by one of its block columns, 0 the substitutions.
template <int KIND>
__global__ __launch_bounds__(NTHR, 2)
void gemm_nn_bf16x3_kernel(int M, int N, int K, const __bf16 *__restrict__ Ah, const __bf16 *__restrict__ Al,
                           int64_t lda, const __bf16 *__restrict__ Bh, const __bf16 *__restrict__ Bl,
                           int64_t ldb, float alpha, float *__restrict__ C, int64_t ldc, const int *skip)
{
    using W = WaveTile<float, TILE>;
    constexpr int BK = Mf<float>::BK;
    constexpr int LDB = KcTile<float>::LDB;
    constexpr int CH = BK / 8;                     // 16-byte chunks per row and stage (4)
    constexpr int PER = TILE * CH / NTHR;          // chunks per thread, per part and operand (2)
    if (skip && *skip) return;
    __shared__ __attribute__((aligned(16))) __bf16 sA[2][2][TILE * LDB];
    __shared__ __attribute__((aligned(16))) __bf16 sB[2][2][TILE * LDB];

    int tm, tn;
    tile_of_block((M + TILE - 1) / TILE, (N + TILE - 1) / TILE, tm, tn);
    const int m0 = tm * TILE, n0 = tn * TILE;
    const int wave = threadIdx.x / CTQR_WAVE;
    const int wn = W::wn(wave), wm = W::wm(wave);

    floatx16 acc[W::NI][W::NJ];
#pragma unroll
    for (int i = 0; i < W::NI; ++i)
#pragma unroll
        for (int j = 0; j < W::NJ; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

    float cpre[W::NI][W::NJ][16];
#pragma unroll
    for (int ib = 0; ib < W::NI; ++ib)
#pragma unroll
        for (int jb = 0; jb < W::NJ; ++jb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int n, m;
                acc_coords<float>(ib, jb, r, n, m);
                n += n0 + wn;
                m += m0 + wm;
                cpre[ib][jb][r] = (m < M && n < N) ? __builtin_nontemporal_load(C + (int64_t)n * ldc + m) : 0.0f;
            }

    bf16x8 ra[2][PER], rb[2][PER];
    auto load = [&](int k) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int f = (int)threadIdx.x + NTHR * q, r = f / CH, c = f % CH;
            const int64_t oa = (int64_t)(m0 + r) * lda + k + 8 * c;
            const int64_t ob = (int64_t)(n0 + r) * ldb + k + 8 * c;
            ra[0][q] = *reinterpret_cast<const bf16x8 *>(Ah + oa);
            ra[1][q] = *reinterpret_cast<const bf16x8 *>(Al + oa);
            rb[0][q] = *reinterpret_cast<const bf16x8 *>(Bh + ob);
            rb[1][q] = *reinterpret_cast<const bf16x8 *>(Bl + ob);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int f = (int)threadIdx.x + NTHR * q, r = f / CH, c = f % CH;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                *reinterpret_cast<bf16x8 *>(&sA[buf][p][r * LDB + 8 * c]) = ra[p][q];
                *reinterpret_cast<bf16x8 *>(&sB[buf][p][r * LDB + 8 * c]) = rb[p][q];
            }
        }
    };
    load(0);
    store(0);
    __syncthreads();
    int cur = 0;
    for (int k = 0; k < K; k += BK) {
        const bool more = k + BK < K;
        if (more) load(k + BK);
        mfma_step_bf2<W::NI, W::NJ>(sB[cur][0], sB[cur][1], sA[cur][0], sA[cur][1], wn, wm, acc);
        if (more) store(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }

#pragma unroll
    for (int ib = 0; ib < W::NI; ++ib)
#pragma unroll
        for (int jb = 0; jb < W::NJ; ++jb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int n, m;
                acc_coords<float>(ib, jb, r, n, m);
                n += n0 + wn;
                m += m0 + wm;
                if (m < M && n < N)
                    __builtin_nontemporal_store(cpre[ib][jb][r] + alpha * acc[ib][jb][r], C + (int64_t)n * ldc + m);
            }
}

// The same product on 256 x 256 output tiles: 8 waves (two per SIMD), each
// a 128-row x 64-column sub-tile (4 x 2 MFMA blocks), two LDS stages of
// 2 x 2 x 256 rows x 32 k in the swizzled layout (swz_off; 128 KiB, dynamic).
// Per 16-deep k step a wave reads 12 KiB of fragments for 24 MFMAs (the
// 128 x 128 tile: 8 KiB for 12).  Every output sums the same products in the
// same order as gemm_nn_bf16x3_kernel, so the two give the same bits.  C is
// read in the epilogue (the staging and fragment registers are free by then).
// Operands are padded to whole 256-row (column) tiles.
constexpr int BIGT = 256;       // output tile edge of the 8-wave form
constexpr int BIGTHR = 512;     // its threads
constexpr int BIG_LDS = 2 * 2 * 2 * BIGT * 32 * 2;   // bytes: stages x operands x parts x rows x 32 k

__global__ __launch_bounds__(BIGTHR, 1)
void gemm_nn_bf16x3_w8_kernel(int M, int N, int K, const __bf16 *__restrict__ Ah, const __bf16 *__restrict__ Al,
                              int64_t lda, const __bf16 *__restrict__ Bh, const __bf16 *__restrict__ Bl,
                              int64_t ldb, float alpha, float *__restrict__ C, int64_t ldc, const int *skip)
{
    constexpr int BK = Mf<float>::BK;
    constexpr int LDB = 32;                        // swizzled rows, no padding
    constexpr int CH = BK / 8;                     // 16-byte chunks per row and stage (4)
    constexpr int PER = BIGT * CH / BIGTHR;        // chunks per thread, per part and operand (2)
    constexpr int NI = 2, NJ = 4;                  // MFMA blocks: output columns, output rows
    constexpr int STAGE = 2 * BIGT * LDB;          // elements of one operand's two parts
    static_assert(BK == 32 && BIG_LDS == 2 * 2 * STAGE * 2, "LDS layout");
    if (skip && *skip) return;
    extern __shared__ __attribute__((aligned(16))) __bf16 big_lds[];
    __bf16 *sA = big_lds;                          // [stage][part][row][k]
    __bf16 *sB = big_lds + 2 * STAGE;              // [stage][part][col][k]

    int tm, tn;
    tile_of_block((M + BIGT - 1) / BIGT, (N + BIGT - 1) / BIGT, tm, tn);
    const int m0 = tm * BIGT, n0 = tn * BIGT;
    const int wave = threadIdx.x / CTQR_WAVE;
    const int wm = (wave % 2) * 128, wn = (wave / 2) * 64;

    floatx16 acc[NI][NJ];
#pragma unroll
    for (int i = 0; i < NI; ++i)
#pragma unroll
        for (int j = 0; j < NJ; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

    bf16x8 ra[2][PER], rb[2][PER];
    auto load = [&](int k) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int f = (int)threadIdx.x + BIGTHR * q, r = f / CH, c = f % CH;
            const int64_t oa = (int64_t)(m0 + r) * lda + k + 8 * c;
            const int64_t ob = (int64_t)(n0 + r) * ldb + k + 8 * c;
            ra[0][q] = *reinterpret_cast<const bf16x8 *>(Ah + oa);
            ra[1][q] = *reinterpret_cast<const bf16x8 *>(Al + oa);
            rb[0][q] = *reinterpret_cast<const bf16x8 *>(Bh + ob);
            rb[1][q] = *reinterpret_cast<const bf16x8 *>(Bl + ob);
        }
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int f = (int)threadIdx.x + BIGTHR * q, r = f / CH, c = f % CH;
#pragma unroll
            for (int p = 0; p < 2; ++p) {
                *reinterpret_cast<bf16x8 *>(&sA[buf * STAGE + p * BIGT * LDB + swz_off(r, c)]) = ra[p][q];
                *reinterpret_cast<bf16x8 *>(&sB[buf * STAGE + p * BIGT * LDB + swz_off(r, c)]) = rb[p][q];
            }
        }
    };
    load(0);
    store(0);
    __syncthreads();
    int cur = 0;
    for (int k = 0; k < K; k += BK) {
        const bool more = k + BK < K;
        if (more) load(k + BK);
        const __bf16 *b0 = sB + cur * STAGE, *a0 = sA + cur * STAGE;
        mfma_step_bf2_swz<NI, NJ>(b0, b0 + BIGT * LDB, a0, a0 + BIGT * LDB, wn, wm, acc);
        if (more) store(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }

    // C += alpha acc, one block column (ib) at a time: its loads first, then
    // its stores
#pragma unroll
    for (int ib = 0; ib < NI; ++ib) {
        float cv[NJ][16];
#pragma unroll
        for (int jb = 0; jb < NJ; ++jb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int n, m;
                acc_coords<float>(ib, jb, r, n, m);
                n += n0 + wn;
                m += m0 + wm;
                cv[jb][r] = (m < M && n < N) ? __builtin_nontemporal_load(C + (int64_t)n * ldc + m) : 0.0f;
            }
#pragma unroll
        for (int jb = 0; jb < NJ; ++jb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int n, m;
                acc_coords<float>(ib, jb, r, n, m);
                n += n0 + wn;
                m += m0 + wm;
                if (m < M && n < N)
                    __builtin_nontemporal_store(cv[jb][r] + alpha * acc[ib][jb][r], C + (int64_t)n * ldc + m);
            }
    }
}

// V (rows x kc Householder block, column-major) to high / low bf16 parts in
// its own column-major layout (k = row contiguous), column stride ldk; rows
// up to ldk and columns up to cols_pad are zero.  These are the A operand of
// the split-BF16 reduction [G | W] = V^T [V | C].  Thread: one column, 8
// consecutive rows.
__global__ __launch_bounds__(256)
void split_vt_kernel(int rows, int kc, const float *__restrict__ V, int64_t lda, int ldk, int cols_pad,
                     __bf16 *__restrict__ hi, __bf16 *__restrict__ lo, int mask, const int *skip)
{
    if (skip && *skip) return;
    const int groups = ldk / 8;
    const int64_t f = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (f >= (int64_t)cols_pad * groups) return;
    const int c = (int)(f / groups), r0 = 8 * (int)(f % groups);
    float xs[8];
    const float *p = V + (int64_t)c * lda + r0;
    if (c < kc && r0 + 8 <= rows && ((uintptr_t)p & 15) == 0) {
        // whole chunk in range: two 16-byte loads
        const floatx4 a0 = *reinterpret_cast<const floatx4 *>(p);
        const floatx4 a1 = *reinterpret_cast<const floatx4 *>(p + 4);
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            xs[e] = a0[e];
            xs[4 + e] = a1[e];
        }
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e) xs[e] = (r0 + e < rows && c < kc) ? p[e] : 0.0f;
    }
    bf16x8 oh, ol;
#pragma unroll
    for (int e = 0; e < 8; ++e) {
        const int r = r0 + e;
        float x = xs[e];
        if (mask && r < rows && c < kc) x = vmask(x, r, c);
        const __bf16 t = (__bf16)x;
        oh[e] = t;
        ol[e] = (__bf16)(x - (float)t);
    }
    *reinterpret_cast<bf16x8 *>(hi + (int64_t)c * ldk + r0) = oh;
    *reinterpret_cast<bf16x8 *>(lo + (int64_t)c * ldk + r0) = ol;
}

// Out = alpha A^T B + beta Out (or split-K partials) with A given as split
// parts (Ah / Al, [col][k], column stride ldk, zero-padded) and B an FP32
// operand split while staged, as gemm_tn_kernel<float, 128, 2>: the same
// products in the same order, without re-splitting A in every column tile.
__global__ __launch_bounds__(NTHR, 2)
void gemm_tn_bf16x3_kernel(int M, int N, int K, const __bf16 *__restrict__ Ah, const __bf16 *__restrict__ Al,
                           int64_t ldk, const float *__restrict__ B, int64_t ldb, int bmask, float alpha, float beta,
                           float *__restrict__ Out, int64_t ldo, float *__restrict__ part, int kchunk, const int *skip,
                           int gram_cols)
{
    using W = WaveTile<float, TILE>;
    constexpr int BK = Mf<float>::BK;
    constexpr int LDB = KcTile<float>::LDB;
    constexpr int CH = BK / 8;
    constexpr int PER = TILE * CH / NTHR;
    if (skip && *skip) return;
    __shared__ __attribute__((aligned(16))) __bf16 sA[2][2][TILE * LDB];
    __shared__ __attribute__((aligned(16))) __bf16 sB[2][2][TILE * LDB];

    int tm, tn;
    tile_of_block((M + TILE - 1) / TILE, (N + TILE - 1) / TILE, tm, tn);
    const int m0 = tm * TILE, n0 = tn * TILE;
    // the first gram_cols output columns are the symmetric Gram V^T V, read
    // only on and above its diagonal: tiles wholly below it are not formed
    if (n0 + TILE <= gram_cols && n0 + TILE <= m0) return;
    const int kbeg = blockIdx.z * kchunk;
    const int kend = min(K, kbeg + kchunk);
    const int wave = threadIdx.x / CTQR_WAVE;
    const int wn = W::wn(wave), wm = W::wm(wave);

    floatx16 acc[W::NI][W::NJ];
#pragma unroll
    for (int i = 0; i < W::NI; ++i)
#pragma unroll
        for (int j = 0; j < W::NJ; ++j)
#pragma unroll
            for (int e = 0; e < 16; ++e) acc[i][j][e] = 0.0f;

    bf16x8 ra[2][PER];
    KcTile<float> lb;
    auto load = [&](int k) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int f = (int)threadIdx.x + NTHR * q, c = f / CH, h = f % CH;
            const int64_t o = (int64_t)(m0 + c) * ldk + k + 8 * h;
            ra[0][q] = *reinterpret_cast<const bf16x8 *>(Ah + o);
            ra[1][q] = *reinterpret_cast<const bf16x8 *>(Al + o);
        }
        lb.load(B, ldb, N, n0, k, kend, bmask);
    };
    auto store = [&](int buf) {
#pragma unroll
        for (int q = 0; q < PER; ++q) {
            const int f = (int)threadIdx.x + NTHR * q, c = f / CH, h = f % CH;
            *reinterpret_cast<bf16x8 *>(&sA[buf][0][c * LDB + 8 * h]) = ra[0][q];
            *reinterpret_cast<bf16x8 *>(&sA[buf][1][c * LDB + 8 * h]) = ra[1][q];
        }
        lb.store_bf2(sB[buf][0], sB[buf][1]);
    };
    if (kbeg < kend) {
        load(kbeg);
        store(0);
    }
    __syncthreads();
    int cur = 0;
    for (int k = kbeg; k < kend; k += BK) {
        const bool more = k + BK < kend;
        if (more) load(k + BK);
        mfma_step_bf2<W::NI, W::NJ>(sB[cur][0], sB[cur][1], sA[cur][0], sA[cur][1], wn, wm, acc);
        if (more) store(cur ^ 1);
        __syncthreads();
        cur ^= 1;
    }

    const bool split = gridDim.z > 1;
#pragma unroll
    for (int ib = 0; ib < W::NI; ++ib)
#pragma unroll
        for (int jb = 0; jb < W::NJ; ++jb)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                int n, m;
                acc_coords<float>(ib, jb, r, n, m);
                n += n0 + wn;
                m += m0 + wm;
                if (m < M && n < N) {
                    const float v = acc[ib][jb][r];
                    if (split) {
                        part[((int64_t)blockIdx.z * N + n) * M + m] = v;
                    } else {
                        float *o = Out + (int64_t)n * ldo + m;
                        *o = beta == 0.0f ? alpha * v : alpha * v + beta * *o;
                    }
                }
            }
}

int g_num_cus = 0;

int num_cus()
{
    if (g_num_cus == 0) {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            g_num_cus = p.multiProcessorCount;
        else
            g_num_cus = 256;
    }
    return g_num_cus;
}

}  // namespace

// ---------------------------------------------------------------------------
// Host launchers
// ---------------------------------------------------------------------------
namespace {
// Products with at most this many output columns use the 128 x 32 tile
// (per host thread; 0 = always the 128 x 128 tile).
thread_local int t_narrow_max = 0;
constexpr int NARROW = 32;
}  // namespace

int gemm_narrow_max() { return t_narrow_max; }
void gemm_set_narrow_max(int n) { t_narrow_max = n < 0 ? 0 : n; }

size_t gemm_tn_partial_elems(int M, int N, int K)
{
    int splits = gemm_tn_splits(M, N, K);
    return splits > 1 ? (size_t)splits * M * N : 0;
}

int gemm_tn_splits(int M, int N, int K)
{
    const bool narrow = N <= t_narrow_max;
    int64_t tiles = ceil_div(M, TILE) * ceil_div(N, narrow ? NARROW : TILE);
    int target = 2 * num_cus();
    if (tiles >= target) return 1;
    int64_t splits = ceil_div(target, tiles);
    int64_t max_by_k = K / (4 * 32);   // keep at least 4 k-steps per split
    if (splits > max_by_k) splits = max_by_k;
    if (splits < 1) splits = 1;
    // products with few output tiles read tall operands (the inner-panel
    // reductions V^T C of a 32-wide panel, Q^T B of few slices): up to 256
    // splits, so the read still spreads over every CU
    if (splits > 256) splits = 256;
    return (int)splits;
}

// Out = alpha * sum of the split partials + beta * Out.  Many splits (a tall,
// narrow product): 16 waves share each output group.  The choice depends on
// the split count only, so products that differ only in their number of
// columns within one column tile sum every output in the same order.
template <typename T>
ctqr_status splitk_reduce(int M, int N, int splits, const T *part, T alpha, T beta, T *Out, int64_t ldo,
                          const int *skip, hipStream_t st)
{
    const int64_t groups = ceil_div((int64_t)M * N, 64);
    if (splits >= 64)
        LAUNCH_TRY((splitk_reduce_kernel<T, 16>), dim3((unsigned)groups), dim3(64 * 16), 0, st, M, N, splits,
                   part, alpha, beta, Out, ldo, skip);
    else
        LAUNCH_TRY((splitk_reduce_kernel<T, 4>), dim3((unsigned)groups), dim3(64 * 4), 0, st, M, N, splits,
                   part, alpha, beta, Out, ldo, skip);
    return CTQR_OK;
}

template <typename T>
ctqr_status gemm_tn(int M, int N, int K, const T *A, int64_t lda, int amask, const T *B,
                    int64_t ldb, int bmask, T alpha, T beta, T *Out, int64_t ldo, T *part,
                    size_t part_elems, const int *skip, hipStream_t st, int force_splits, int bf16, int tri)
{
    if (M <= 0 || N <= 0) return CTQR_OK;
    if (bf16 == 2) return CTQR_EINVAL;   // split operands: gemm_tn_bf16x3
    if (tri < 0 || tri > 2 || (tri != 0 && M != K)) return CTQR_EINVAL;
    const bool narrow = N <= t_narrow_max;
    int splits = force_splits > 0 ? force_splits : gemm_tn_splits(M, N, K);
    if (splits > 1 && (part == nullptr || part_elems < (size_t)splits * M * N)) {
        if (force_splits > 0) return CTQR_ENOMEM;   // a forced split must not silently change
        splits = 1;
    }
    int kchunk = (int)ceil_div(ceil_div(K, splits), Mf<T>::BK) * Mf<T>::BK;
    if (kchunk <= 0) kchunk = Mf<T>::BK;
    splits = (int)ceil_div(K > 0 ? K : 1, kchunk);
    dim3 grid((unsigned)(ceil_div(M, TILE) * ceil_div(N, narrow ? NARROW : TILE)), 1, (unsigned)splits);
    bool done = false;
    if constexpr (sizeof(T) == 4) {
        if (bf16 == 1 && !narrow) {
            LAUNCH_TRY((gemm_tn_kernel<T, TILE, 1>), grid, dim3(NTHR), 0, st, M, N, K, A, lda, amask, B, ldb,
                       bmask, alpha, beta, Out, ldo, part, kchunk, skip, tri);
            done = true;
        }
    }
    if (done) {
    } else if (narrow) {
        LAUNCH_TRY((gemm_tn_kernel<T, NARROW, 0>), grid, dim3(NTHR), 0, st, M, N, K, A, lda, amask, B, ldb,
                   bmask, alpha, beta, Out, ldo, part, kchunk, skip, tri);
    } else {
        LAUNCH_TRY((gemm_tn_kernel<T, TILE, 0>), grid, dim3(NTHR), 0, st, M, N, K, A, lda, amask, B, ldb,
                   bmask, alpha, beta, Out, ldo, part, kchunk, skip, tri);
    }
    if (splits > 1) return splitk_reduce<T>(M, N, splits, part, alpha, beta, Out, ldo, skip, st);
    return CTQR_OK;
}

template <typename T>
ctqr_status gemm_tn_tprod(int M, int N, int K, const T *A, int64_t lda, int amask, const T *B, int64_t ldb,
                          const T *Tt, int64_t ldt, T *Out, int64_t ldo, T *W2, int64_t ldw, T *part,
                          size_t part_elems, hipStream_t st)
{
    if (M <= 0 || N <= 0) return CTQR_OK;
    if (M > 32) return CTQR_EINVAL;
    int splits = gemm_tn_splits(M, N, K);
    if (splits > 1 && (part == nullptr || part_elems < (size_t)splits * M * N)) splits = 1;
    int kchunk = (int)ceil_div(ceil_div(K, splits), Mf<T>::BK) * Mf<T>::BK;
    if (kchunk <= 0) kchunk = Mf<T>::BK;
    splits = (int)ceil_div(K > 0 ? K : 1, kchunk);
    // A^T B formed as B^T A on the 128 x 32 tile (no output rows padded from
    // M to 128), written transposed into A^T B's places
    dim3 grid((unsigned)ceil_div(N, TILE), 1, (unsigned)splits);
    LAUNCH_TRY((gemm_tn_kernel<T, NARROW, 0, true>), grid, dim3(NTHR), 0, st, N, M, K, B, ldb, 0, A, lda, amask,
               T(1), T(0), Out, ldo, part, kchunk, (const int *)nullptr, 0);
    const bool sp = splits > 1;
    LAUNCH_TRY(tprod_reduce_kernel<T>, dim3((unsigned)ceil_div(N, 2)), dim3(1024), 0, st, M, N, splits,
               sp ? (const T *)part : (const T *)Out, sp ? (int64_t)M : ldo, (int64_t)M * N, Tt, ldt, W2, ldw);
    return CTQR_OK;
}

template <typename T>
ctqr_status gemm_nn(int M, int N, int K, const T *A, int64_t lda, int amask, const T *B,
                    int64_t ldb, T alpha, T *C, int64_t ldc, const int *skip, hipStream_t st, int kind,
                    int accum, int bf16)
{
    if (M <= 0 || N <= 0) return CTQR_OK;
    if (bf16 == 2) return CTQR_EINVAL;   // split operands: gemm_nn_bf16x3
    if (K <= 0) {
        if (accum) return CTQR_OK;
        K = 0;   // C = 0: the kernel runs with an empty k loop
    }
    const bool narrow = N <= t_narrow_max;
    const int kchunk = K > 0 ? K : 1;
    dim3 grid((unsigned)(ceil_div(M, TILE) * ceil_div(N, narrow ? NARROW : TILE)));
    if constexpr (sizeof(T) == 4) {
        if (kind == 1 && bf16 == 1) {
            LAUNCH_TRY((gemm_nn_kernel<T, 1, TILE, false, 1>), grid, dim3(NTHR), 0, st, M, N, K, A, lda, amask,
                       B, ldb, alpha, C, ldc, accum, (T *)nullptr, kchunk, skip, (int64_t)0, (int64_t)0,
                       (int64_t)0);
            return CTQR_OK;
        }

    }
    if (kind == 1)
        LAUNCH_TRY((gemm_nn_kernel<T, 1, TILE, false, 0>), grid, dim3(NTHR), 0, st, M, N, K, A, lda, amask, B,
                   ldb, alpha, C, ldc, accum, (T *)nullptr, kchunk, skip, (int64_t)0, (int64_t)0, (int64_t)0);
    else if (narrow)
        LAUNCH_TRY((gemm_nn_kernel<T, 0, NARROW, false, 0>), grid, dim3(NTHR), 0, st, M, N, K, A, lda, amask,
                   B, ldb, alpha, C, ldc, accum, (T *)nullptr, kchunk, skip, (int64_t)0, (int64_t)0, (int64_t)0);
    else
        LAUNCH_TRY((gemm_nn_kernel<T, 0, TILE, false, 0>), grid, dim3(NTHR), 0, st, M, N, K, A, lda, amask,
                   B, ldb, alpha, C, ldc, accum, (T *)nullptr, kchunk, skip, (int64_t)0, (int64_t)0, (int64_t)0);
    return CTQR_OK;
}

template <typename T>
ctqr_status gemm_nn_batched(int M, int N, int K, const T *A, int64_t lda, int64_t bsa, const T *B, int64_t ldb,
                            int64_t bsb, T alpha, T *C, int64_t ldc, int64_t bsc, int batch, int accum,
                            hipStream_t st)
{
    if (M <= 0 || N <= 0 || K <= 0 || batch <= 0) return CTQR_OK;
    if (batch > 65535) return CTQR_EINVAL;
    const bool narrow = N <= t_narrow_max;
    dim3 grid((unsigned)(ceil_div(M, TILE) * ceil_div(N, narrow ? NARROW : TILE)), (unsigned)batch);
    if (narrow)
        LAUNCH_TRY((gemm_nn_kernel<T, 0, NARROW, false, 0>), grid, dim3(NTHR), 0, st, M, N, K, A, lda, 0, B, ldb,
                   alpha, C, ldc, accum, (T *)nullptr, K, (const int *)nullptr, bsa, bsb, bsc);
    else
        LAUNCH_TRY((gemm_nn_kernel<T, 0, TILE, false, 0>), grid, dim3(NTHR), 0, st, M, N, K, A, lda, 0, B, ldb,
                   alpha, C, ldc, accum, (T *)nullptr, K, (const int *)nullptr, bsa, bsb, bsc);
    return CTQR_OK;
}

template <typename T>
ctqr_status gemm_nn_split(int M, int N, int K, const T *A, int64_t lda, const T *B, int64_t ldb, T alpha,
                          T *C, int64_t ldc, T *part, size_t part_elems, const int *skip, hipStream_t st)
{
    if (M <= 0 || N <= 0 || K <= 0) return CTQR_OK;
    const bool narrow = N <= t_narrow_max;
    int splits = gemm_tn_splits(M, N, K);
    if (splits > 1 && (part == nullptr || part_elems < (size_t)splits * M * N)) splits = 1;
    if (splits <= 1) return gemm_nn<T>(M, N, K, A, lda, 0, B, ldb, alpha, C, ldc, skip, st, 0, 1, 0);
    int kchunk = (int)ceil_div(ceil_div(K, splits), Mf<T>::BK) * Mf<T>::BK;
    splits = (int)ceil_div(K, kchunk);
    dim3 grid((unsigned)(ceil_div(M, TILE) * ceil_div(N, narrow ? NARROW : TILE)), 1, (unsigned)splits);
    if (narrow)
        LAUNCH_TRY((gemm_nn_kernel<T, 0, NARROW, true, 0>), grid, dim3(NTHR), 0, st, M, N, K, A, lda, 0, B,
                   ldb, alpha, C, ldc, 0, part, kchunk, skip, (int64_t)0, (int64_t)0, (int64_t)0);
    else
        LAUNCH_TRY((gemm_nn_kernel<T, 0, TILE, true, 0>), grid, dim3(NTHR), 0, st, M, N, K, A, lda, 0, B,
                   ldb, alpha, C, ldc, 0, part, kchunk, skip, (int64_t)0, (int64_t)0, (int64_t)0);
    return splitk_reduce<T>(M, N, splits, part, alpha, T(1), C, ldc, skip, st);
}

namespace {
int64_t up_to(int64_t a, int64_t b) { return ceil_div(a, b) * b; }
}  // namespace

size_t bf16x3_split_elems(int64_t m, int64_t n, int nb)
{
    const int64_t kp = up_to(nb, 32);
    return (size_t)(2 * up_to(m, BIGT) * kp + 2 * up_to(n, BIGT) * kp);
}

namespace {
// the 8-wave form of the trailing update (CTQR_GEMM_W8=0 keeps the 128 x 128 one)
bool w8_enabled()
{
    const char *e = std::getenv("CTQR_GEMM_W8");
    return !(e && e[0] == '0');
}

struct SplitParts {
    int kp, rows_pad, cols_pad;
    __bf16 *vh, *vl, *wh, *wl;
};
bool split_parts(int M, int N, int K, __bf16 *split, size_t split_elems, SplitParts &p)
{
    p.kp = (int)up_to(K, 32);
    p.rows_pad = (int)up_to(M, BIGT);           // whole tiles of either update kernel
    p.cols_pad = (int)up_to(N, BIGT);
    const size_t need = 2 * (size_t)p.rows_pad * p.kp + 2 * (size_t)p.cols_pad * p.kp;
    if (split == nullptr || need > split_elems) return false;
    p.vh = split;
    p.vl = p.vh + (size_t)p.rows_pad * p.kp;
    p.wh = p.vl + (size_t)p.rows_pad * p.kp;
    p.wl = p.wh + (size_t)p.cols_pad * p.kp;
    return true;
}
}  // namespace

ctqr_status bf16x3_split(int M, int N, int K, const float *V, int64_t lda, const float *W, int64_t ldw,
                         __bf16 *split, size_t split_elems, hipStream_t st, bool householder, const int *skip)
{
    if (M <= 0 || N <= 0 || K <= 0) return CTQR_OK;
    SplitParts p;
    if (!split_parts(M, N, K, split, split_elems, p)) return CTQR_ENOMEM;
    LAUNCH_TRY(split_v_kernel, dim3((unsigned)ceil_div(p.rows_pad, SPLIT_V_T), (unsigned)ceil_div(p.kp, SPLIT_V_T)),
               dim3(256), 0, st, M, K, V, lda, p.rows_pad, p.kp, p.vh, p.vl, householder ? 1 : 0, skip);
    LAUNCH_TRY(split_w_kernel, dim3((unsigned)ceil_div((int64_t)p.cols_pad * (p.kp / 8), 256)), dim3(256), 0, st, K,
               N, W, ldw, p.cols_pad, p.kp, p.wh, p.wl, skip);
    return CTQR_OK;
}

size_t bf16x3_vt_elems(int64_t m, int nb)
{
    return (size_t)(2 * up_to(m, 32) * up_to(nb, TILE));
}

ctqr_status bf16x3_split_vt(int rows, int kc, const float *V, int64_t lda, __bf16 *vt, size_t vt_elems,
                            hipStream_t st, bool householder, const int *skip)
{
    if (rows <= 0 || kc <= 0) return CTQR_OK;
    const int ldk = (int)up_to(rows, 32), cols_pad = (int)up_to(kc, TILE);
    if (vt == nullptr || 2 * (size_t)ldk * cols_pad > vt_elems) return CTQR_ENOMEM;
    LAUNCH_TRY(split_vt_kernel, dim3((unsigned)ceil_div((int64_t)cols_pad * (ldk / 8), 256)), dim3(256), 0, st, rows,
               kc, V, lda, ldk, cols_pad, vt, vt + (size_t)ldk * cols_pad, householder ? 1 : 0, skip);
    return CTQR_OK;
}

ctqr_status gemm_tn_bf16x3(int M, int N, int K, const __bf16 *vt, size_t vt_elems, const float *B, int64_t ldb,
                           int bmask, float alpha, float beta, float *Out, int64_t ldo, float *part,
                           size_t part_elems, const int *skip, hipStream_t st, int force_splits, int gram_cols)
{
    if (M <= 0 || N <= 0) return CTQR_OK;
    const int ldk = (int)up_to(K, 32), cols_pad = (int)up_to(M, TILE);
    if (vt == nullptr || 2 * (size_t)ldk * cols_pad > vt_elems) return CTQR_ENOMEM;
    // the same split rule as gemm_tn (128-wide tiles), so a forced split count
    // sums every output in the same order as there
    const int narrow_saved = t_narrow_max;
    t_narrow_max = 0;
    int splits = force_splits > 0 ? force_splits : gemm_tn_splits(M, N, K);
    t_narrow_max = narrow_saved;
    if (splits > 1 && (part == nullptr || part_elems < (size_t)splits * M * N)) {
        if (force_splits > 0) return CTQR_ENOMEM;
        splits = 1;
    }
    int kchunk = (int)ceil_div(ceil_div(K, splits), Mf<float>::BK) * Mf<float>::BK;
    if (kchunk <= 0) kchunk = Mf<float>::BK;
    splits = (int)ceil_div(K > 0 ? K : 1, kchunk);
    dim3 grid((unsigned)(ceil_div(M, TILE) * ceil_div(N, TILE)), 1, (unsigned)splits);
    LAUNCH_TRY(gemm_tn_bf16x3_kernel, grid, dim3(NTHR), 0, st, M, N, K, vt, vt + (size_t)ldk * cols_pad,
               (int64_t)ldk, B, ldb, bmask, alpha, beta, Out, ldo, part, kchunk, skip, gram_cols);
    if (splits > 1) return splitk_reduce<float>(M, N, splits, part, alpha, beta, Out, ldo, skip, st);
    return CTQR_OK;
}

ctqr_status bf16x3_split_rows(int M, int K, const float *V, int64_t lda, bool householder, __bf16 *hi, __bf16 *lo,
                              int ldp, int rows_pad, hipStream_t st, const int *skip)
{
    if (M <= 0 || K <= 0) return CTQR_OK;
    if (ldp < K || ldp % 8 != 0 || rows_pad < M || rows_pad % TILE != 0) return CTQR_EINVAL;
    LAUNCH_TRY(split_v_kernel, dim3((unsigned)ceil_div(rows_pad, SPLIT_V_T), (unsigned)ceil_div(ldp, SPLIT_V_T)),
               dim3(256), 0, st, M, K, V, lda, rows_pad, ldp, hi, lo, householder ? 1 : 0, skip);
    return CTQR_OK;
}

ctqr_status bf16x3_split_cols(int K, int N, const float *W, int64_t ldw, __bf16 *hi, __bf16 *lo, int ldp,
                              int cols_pad, hipStream_t st, const int *skip)
{
    if (N <= 0 || K <= 0) return CTQR_OK;
    if (ldp < K || ldp % 8 != 0 || cols_pad < N || cols_pad % TILE != 0) return CTQR_EINVAL;
    LAUNCH_TRY(split_w_kernel, dim3((unsigned)ceil_div((int64_t)cols_pad * (ldp / 8), 256)), dim3(256), 0, st, K, N,
               W, ldw, cols_pad, ldp, hi, lo, skip);
    return CTQR_OK;
}

ctqr_status gemm_nn_bf16x3_parts(int M, int N, int K, float alpha, float *C, int64_t ldc, const __bf16 *ah,
                                 const __bf16 *al, int64_t lda_p, const __bf16 *bh, const __bf16 *bl, int64_t ldb_p,
                                 hipStream_t st, const int *skip)
{
    if (M <= 0 || N <= 0 || K <= 0) return CTQR_OK;
    if (lda_p < up_to(K, 32) || ldb_p < up_to(K, 32)) return CTQR_EINVAL;
    dim3 grid((unsigned)(ceil_div(M, TILE) * ceil_div(N, TILE)));
    LAUNCH_TRY(gemm_nn_bf16x3_kernel<0>, grid, dim3(NTHR), 0, st, M, N, K, ah, al, lda_p, bh, bl, ldb_p, alpha, C,
               ldc, skip);
    return CTQR_OK;
}

ctqr_status gemm_nn_bf16x3(int M, int N, int K, float alpha, float *C, int64_t ldc, const __bf16 *split,
                           size_t split_elems, hipStream_t st, const int *skip, int kind)
{
    if (M <= 0 || N <= 0 || K <= 0) return CTQR_OK;
    if (kind != 1 && kind != 2) return CTQR_EINVAL;
    SplitParts p;
    if (!split_parts(M, N, K, const_cast<__bf16 *>(split), split_elems, p)) return CTQR_ENOMEM;
    dim3 grid((unsigned)(ceil_div(M, TILE) * ceil_div(N, TILE)));
    if (kind == 1 && w8_enabled() && (int64_t)ceil_div(M, BIGT) * ceil_div(N, BIGT) >= 2 * 256) {
        static bool attr = false;
        if (!attr) {
            HIP_TRY(hipFuncSetAttribute((const void *)gemm_nn_bf16x3_w8_kernel,
                                        hipFuncAttributeMaxDynamicSharedMemorySize, BIG_LDS));
            attr = true;
        }
        dim3 g8((unsigned)(ceil_div(M, BIGT) * ceil_div(N, BIGT)));
        LAUNCH_TRY(gemm_nn_bf16x3_w8_kernel, g8, dim3(BIGTHR), BIG_LDS, st, M, N, K, (const __bf16 *)p.vh,
                   (const __bf16 *)p.vl, (int64_t)p.kp, (const __bf16 *)p.wh, (const __bf16 *)p.wl, (int64_t)p.kp,
                   alpha, C, ldc, skip);
    } else if (kind == 1)
        LAUNCH_TRY(gemm_nn_bf16x3_kernel<1>, grid, dim3(NTHR), 0, st, M, N, K, (const __bf16 *)p.vh,
                   (const __bf16 *)p.vl, (int64_t)p.kp, (const __bf16 *)p.wh, (const __bf16 *)p.wl, (int64_t)p.kp,
                   alpha, C, ldc, skip);
    else
        LAUNCH_TRY(gemm_nn_bf16x3_kernel<2>, grid, dim3(NTHR), 0, st, M, N, K, (const __bf16 *)p.vh,
                   (const __bf16 *)p.vl, (int64_t)p.kp, (const __bf16 *)p.wh, (const __bf16 *)p.wl, (int64_t)p.kp,
                   alpha, C, ldc, skip);
    return CTQR_OK;
}

template ctqr_status gemm_tn<float>(int, int, int, const float *, int64_t, int, const float *,
                                    int64_t, int, float, float, float *, int64_t, float *, size_t,
                                    const int *, hipStream_t, int, int, int);
template ctqr_status gemm_tn<double>(int, int, int, const double *, int64_t, int, const double *,
                                     int64_t, int, double, double, double *, int64_t, double *,
                                     size_t, const int *, hipStream_t, int, int, int);
template ctqr_status gemm_tn_tprod<float>(int, int, int, const float *, int64_t, int, const float *, int64_t,
                                          const float *, int64_t, float *, int64_t, float *, int64_t, float *,
                                          size_t, hipStream_t);
template ctqr_status gemm_tn_tprod<double>(int, int, int, const double *, int64_t, int, const double *, int64_t,
                                           const double *, int64_t, double *, int64_t, double *, int64_t,
                                           double *, size_t, hipStream_t);
template ctqr_status gemm_nn<float>(int, int, int, const float *, int64_t, int, const float *,
                                    int64_t, float, float *, int64_t, const int *, hipStream_t, int, int, int);
template ctqr_status gemm_nn<double>(int, int, int, const double *, int64_t, int, const double *,
                                     int64_t, double, double *, int64_t, const int *, hipStream_t, int, int, int);
template ctqr_status gemm_nn_batched<float>(int, int, int, const float *, int64_t, int64_t, const float *, int64_t,
                                            int64_t, float, float *, int64_t, int64_t, int, int, hipStream_t);
template ctqr_status gemm_nn_batched<double>(int, int, int, const double *, int64_t, int64_t, const double *,
                                             int64_t, int64_t, double, double *, int64_t, int64_t, int, int,
                                             hipStream_t);
template ctqr_status gemm_nn_split<float>(int, int, int, const float *, int64_t, const float *, int64_t, float,
                                          float *, int64_t, float *, size_t, const int *, hipStream_t);
template ctqr_status gemm_nn_split<double>(int, int, int, const double *, int64_t, const double *, int64_t,
                                           double, double *, int64_t, double *, size_t, const int *, hipStream_t);
