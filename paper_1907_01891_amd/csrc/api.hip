// C ABI of libctqr: argument checking, workspace carving and the host-side
// drivers of the blocked QR factorization and of the multi-slice solve.
#include <mutex>
#include <string>
#include <vector>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <cmath>

#include "common.h"
#include "kernels.h"

// Device scratch of ctqr_qr_solve_slices_noalloc, for callers that cannot
// allocate: one copy per GPU, held until the process ends.  Host code never
// passes this name to a kernel (on the host it is only a stand-in for the
// device symbol); it uses the device address hipGetSymbolAddress returns for
// each device (noalloc_scratch below).
static __device__ __align__(256) unsigned char scratch[CTQR_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr int PANEL_W = 32;             // inner panel width
constexpr int DEFAULT_NB = 256;         // outer block width
constexpr int MAX_PANEL_WG = GB_GROUP * GB_MAX_GROUPS;   // partial-sum slots of the panel kernel
constexpr int64_t SPLIT_PART_ELEMS = 2LL * 512 * 128 * 128;   // split-K partial buffer

thread_local std::string g_last_error;

struct ProfRec {
    hipEvent_t a, b;
    double flops;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof;
std::vector<ProfRec> g_prof_red;   // the [G | W] reductions' products, likewise

// Phase timing (ctqr_profile_enable bit 2): HIP events around the phases of
// a factorization or a direct solve, on the stream they run on (not inside
// graph capture).  Gaps between phases (host synchronisation) count in none.
struct PhaseRec {
    int phase;
    hipEvent_t a, b;
};
bool g_phase_on = false;
std::vector<PhaseRec> g_phase;
thread_local bool t_no_alloc = false;   // inside ctqr_qr_solve_slices_noalloc: no timing events

struct PhaseScope {
    int phase;
    hipStream_t st;
    hipEvent_t a = nullptr;
    PhaseScope(int p, hipStream_t s) : phase(p), st(s)
    {
        if (t_no_alloc) return;
        {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            if (!g_phase_on) return;
        }
        hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
        if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
        if (hipEventCreate(&a) != hipSuccess) {
            a = nullptr;
            return;
        }
        if (hipEventRecord(a, st) != hipSuccess) {
            (void)hipEventDestroy(a);
            a = nullptr;
        }
    }
    ~PhaseScope()
    {
        if (!a) return;
        hipEvent_t b = nullptr;
        if (hipEventCreate(&b) != hipSuccess || hipEventRecord(b, st) != hipSuccess) {
            (void)hipEventDestroy(a);
            if (b) (void)hipEventDestroy(b);
            return;
        }
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_phase.push_back({phase, a, b});
    }
    PhaseScope(const PhaseScope &) = delete;
    PhaseScope &operator=(const PhaseScope &) = delete;
};

bool aligned16(const void *p) { return ((uintptr_t)p & 15u) == 0; }

// Progress hook of the long out-of-core calls: a host function enqueued on
// the stream, so it runs when the GPU has finished the work before it.
std::mutex g_progress_mu;
ctqr_progress_fn g_progress = nullptr;
void *g_progress_user = nullptr;

struct ProgressMsg {
    ctqr_progress_fn fn;
    void *user;
    int32_t stage;
    int64_t done, total;
};

void progress_trampoline(void *p)
{
    ProgressMsg *msg = static_cast<ProgressMsg *>(p);
    msg->fn(msg->stage, msg->done, msg->total, msg->user);
    delete msg;
}

ctqr_status progress_mark(hipStream_t st, int32_t stage, int64_t done, int64_t total)
{
    ctqr_progress_fn fn;
    void *user;
    {
        std::lock_guard<std::mutex> lk(g_progress_mu);
        fn = g_progress;
        user = g_progress_user;
    }
    if (!fn) return CTQR_OK;
    ProgressMsg *msg = new ProgressMsg{fn, user, stage, done, total};
    hipError_t e = hipLaunchHostFunc(st, progress_trampoline, msg);
    if (e != hipSuccess) {
        delete msg;
        ctqr_last_hip_error(e, "hipLaunchHostFunc", __FILE__, __LINE__);
        return CTQR_EHIP;
    }
    return CTQR_OK;
}


int64_t round_up(int64_t a, int64_t b) { return ceil_div(a, b) * b; }

// Bump allocator over the caller's workspace (256-byte aligned pieces).
struct Carve {
    char *base;
    size_t off = 0;
    explicit Carve(void *b) : base((char *)b) {}
    template <typename T>
    T *take(int64_t count)
    {
        off = (size_t)round_up((int64_t)off, 256);
        T *p = base ? (T *)(base + off) : nullptr;
        off += (size_t)count * sizeof(T);
        return p;
    }
};

// Groups of GROUP consecutive block columns share one trailing update: each
// block's reflector updates only the rest of its group, and the group's
// compact-WY reflectors then act on the remaining columns as one block
// reflector of up to GROUP nb columns (Schreiber and Van Loan, the product form
// of Householder blocks), so the trailing update sweeps the remaining columns
// once per group instead of once per block, with an inner dimension of
// GROUP nb.  Only for nb dividing 512: every range boundary of the out-of-core
// factorization (a multiple of 2048, or n) then falls between groups.
constexpr int GROUP = 4;
int group_blocks(int nb) { return 512 % nb == 0 ? GROUP : 1; }
int gw_rows(int nb) { return group_blocks(nb) * nb; }   // rows of [G | W] and W'

template <typename T>
struct FactorWS {
    unsigned *bars;
    double *part, *part2, *gram_part, *gram, *Tw;
    T *Tin, *GW, *W2, *split, *rtmp;
    T *gstore;               // per group: its Gram V^T V (gw_rows square), for its later applications
    __bf16 *bsplit;          // split-BF16 parts of V and W' (FP32 factor only)
    size_t bsplit_elems;
    __bf16 *vtsplit;         // split-BF16 parts of V, column-major, for [G | W]
    size_t vtsplit_elems;
    size_t bytes;
    int bf16 = 0;   // block-column GEMMs ([G | W], trailing update): bf16 parts per operand (0: none)
};

template <typename T>
FactorWS<T> carve_factor(void *work, int64_t m, int64_t n, int nb)
{
    Carve c(work);
    FactorWS<T> w;
    w.bars = c.take<unsigned>((ceil_div(n, PANEL_W) + 1) * GB_WORDS);
    w.part = c.take<double>(MAX_PANEL_WG + 1);
    w.part2 = c.take<double>(2LL * MAX_PANEL_WG * PANEL_XCH_STRIDE);
    w.gram_part = c.take<double>((int64_t)MAX_PANEL_WG * PANEL_W * PANEL_W);
    w.gram = c.take<double>(PANEL_GRAM_ELEMS);
    w.Tw = c.take<double>((int64_t)nb * nb);
    w.Tin = c.take<T>(PANEL_W * PANEL_W);
    const int g = gw_rows(nb);
    w.GW = c.take<T>((int64_t)g * n);
    w.W2 = c.take<T>((int64_t)g * n);
    w.gstore = c.take<T>(group_blocks(nb) > 1 ? ceil_div(n, g) * g * g : 0);
    w.split = c.take<T>(SPLIT_PART_ELEMS);
    w.rtmp = c.take<T>((int64_t)trinv_tmp_elems());
    w.bsplit_elems = sizeof(T) == 4 ? bf16x3_split_elems(m, n, g) : 0;
    w.bsplit = c.take<__bf16>((int64_t)w.bsplit_elems);
    w.vtsplit_elems = sizeof(T) == 4 ? bf16x3_vt_elems(m, g) : 0;
    w.vtsplit = c.take<__bf16>((int64_t)w.vtsplit_elems);
    w.bytes = c.off + 256;
    return w;
}

template <typename T>
struct SolveWS {
    T *Bw, *W, *W2, *split, *Rinv, *RinvT, *Xw;
    double *xr, *Br, *r, *s, *hist;
    double *xs, *xbest;      // refinement: the iterate before the last update, and the best one kept
    // conjugate-gradient form: z (two, by iteration parity), p, q, dot partials, per-slice scalars
    double *z0, *z1, *p, *q, *dpart, *sz, *szp, *qq, *gamma, *beta, *alpha;
    T *s32, *y32, *d32;
    __bf16 *rparts;          // split-BF16 parts of R for the refinement's wide substitutions (or null)
    __bf16 *xparts;          // and of their right-hand sides (or null)
    __bf16 *qsplit;          // split-BF16 parts of a block of V and of W' for Q^T B (with xparts)
    size_t qsplit_elems;
    unsigned long long *dmax, *xmax, *smax;
    double *s0;
    int *done;
    T *fex;                  // exchange area of the persistent kernels (few slices), or null
    unsigned *fbar;          // and their grid-barrier words
    int64_t ldbw, ldxw;
    size_t bytes;
};

// The wide substitutions of the corrected semi-normal-equations refinement
// take split-BF16 products (all-in-HBM FP32 factor, at least 128 slices, R's
// parts within TRSM_SPLIT_MAX_BYTES):
// each correction only has to contract the error, which an inexact
// (R^T R)^-1 does.  The conjugate-gradient form (refine 2) keeps FP32
// products: it needs the preconditioner to be the same symmetric operator
// in every iteration, and the split products' rounding erodes conjugacy
// before its tolerance is met.
// R's parts take about 4 n^2 bytes (both layouts), so they are used up to a
// fixed size: 32 GiB, n up to about 92,000 (16.6 GB at 256^2).
constexpr size_t TRSM_SPLIT_MAX_BYTES = (size_t)32 << 30;
template <typename T>
bool refine_split_trsm(int64_t n, int S, int refine)
{
    return sizeof(T) == 4 && refine == 1 && S >= TRSM_SPLIT_MIN_SLICES &&
           trsm_rparts_elems(n) * sizeof(__bf16) <= TRSM_SPLIT_MAX_BYTES;
}

// refine: 0 none, 1 semi-normal-equations corrections, 2 also the
// conjugate-gradient vectors; trsm_split: room for those split products
// (TRSM_PARTS_X: the right-hand sides' parts only, R's are elsewhere;
// TRSM_PARTS_ALL: R's parts too).
constexpr int TRSM_PARTS_NONE = 0, TRSM_PARTS_X = 1, TRSM_PARTS_ALL = 2;
template <typename T>
SolveWS<T> carve_solve(void *work, int64_t m, int64_t n, int nb, int S, int refine, bool with_rinv = true,
                       int trsm_split = TRSM_PARTS_NONE)
{
    Carve c(work);
    SolveWS<T> w{};
    w.ldbw = round_up(m, 4);
    w.ldxw = round_up(n, 4);
    w.Bw = c.take<T>(w.ldbw * S);
    w.W = c.take<T>((int64_t)nb * S);
    w.W2 = c.take<T>((int64_t)nb * S);
    int64_t sp = std::max<int64_t>(SPLIT_PART_ELEMS, 64LL * nb * S);
    w.split = c.take<T>(sp);
    if (with_rinv) {   // used when the factor has no stored inverses
        w.Rinv = c.take<T>(2 * (int64_t)trinv_elems((int)n));
        w.RinvT = c.take<T>((int64_t)trinv_tmp_elems());   // scratch of the inverse doubling
    }
    w.Xw = c.take<T>(w.ldxw * S);
    w.done = c.take<int>(64);
    if (S <= FUSED_MAX_S) {
        w.fex = c.take<T>((int64_t)fused_exchange_elems());
        w.fbar = c.take<unsigned>(GB_WORDS);
    }
    if (refine) {
        w.xr = c.take<double>(n * S);
        w.Br = c.take<double>(m * S);
        w.r = c.take<double>(m * S);
        w.s = c.take<double>(n * S);
        w.s32 = c.take<T>(w.ldxw * S);
        w.y32 = c.take<T>(w.ldxw * S);
        w.d32 = c.take<T>(w.ldxw * S);
        w.dmax = c.take<unsigned long long>(S);
        w.xmax = c.take<unsigned long long>(S);
        w.smax = c.take<unsigned long long>(S);
        w.s0 = c.take<double>(S);
        w.hist = c.take<double>(8);
        w.xs = c.take<double>(n * S);
        w.xbest = c.take<double>(n * S);
        const bool parts = trsm_split != TRSM_PARTS_NONE && refine_split_trsm<T>(n, S, refine);
        w.xparts = parts ? c.take<__bf16>((int64_t)trsm_xparts_elems(S)) : nullptr;
        w.qsplit_elems = parts ? bf16x3_split_elems(m, S, nb) : 0;
        w.qsplit = parts ? c.take<__bf16>((int64_t)w.qsplit_elems) : nullptr;
        w.rparts = parts && trsm_split == TRSM_PARTS_ALL ? c.take<__bf16>((int64_t)trsm_rparts_elems(n)) : nullptr;
    }
    if (refine >= 2) {
        w.z0 = c.take<double>(n * S);
        w.z1 = c.take<double>(n * S);
        w.p = c.take<double>(n * S);
        w.q = c.take<double>(m * S);
        w.dpart = c.take<double>((int64_t)slice_dot_partial_elems(S));
        w.sz = c.take<double>(S);
        w.szp = c.take<double>(S);
        w.qq = c.take<double>(S);
        w.gamma = c.take<double>(S);
        w.beta = c.take<double>(S);
        w.alpha = c.take<double>(S);
    }
    w.bytes = c.off + 256;
    return w;
}

int device_cus()
{
    static int cus = 0;
    if (!cus) {
        int dev = 0;
        hipDeviceProp_t p;
        if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&p, dev) == hipSuccess)
            cus = p.multiProcessorCount;
        if (cus <= 0) cus = 256;
    }
    return cus;
}

// Per-thread pinned word the refinement loop reads its convergence flag into.
// Every word is also listed process-wide, so ctqr_release can free them all.
std::mutex g_flags_mu;
std::vector<int *> g_flags;
uint64_t g_flags_epoch = 0;   // bumped by ctqr_release: cached words are stale

int *host_flag()
{
    thread_local int *p = nullptr;
    thread_local uint64_t epoch = 0;
    std::lock_guard<std::mutex> lk(g_flags_mu);
    if (p && epoch != g_flags_epoch) p = nullptr;
    if (!p) {
        if (hipHostMalloc((void **)&p, 64, hipHostMallocDefault) != hipSuccess) return p = nullptr;
        g_flags.push_back(p);
        epoch = g_flags_epoch;
    }
    return p;
}

ctqr_status ensure_setup()
{
    static std::once_flag once;
    static ctqr_status st = CTQR_OK;
    std::call_once(once, [] { st = panel_setup(panel_max_rows_per_wg()); });
    return st;
}

// Profiled launch of the trailing update C -= V W' (the dominant kernel).
// C -= V W' (V: mk x nbk Householder block, W': nbk x nc, column stride nb).
// partner: the update of the rest of a group of block columns by one of its
// blocks, launched as its own kernel instance (FP32 MFMA in the one-part BF16
// mode) and left out of the profile records, which hold the trailing updates
// only.
template <typename T>
ctqr_status trailing_update(int mk, int nc, int nbk, const T *V, int64_t lda, const T *W2, int nb, T *C,
                            hipStream_t st, int bf16, __bf16 *bsplit, size_t bsplit_elems, bool partner = false)
{
    if constexpr (sizeof(T) == 4) {
        // split-BF16: both operands split once, outside the timed product
        if (bf16 == 2) {
            ctqr_status s = bf16x3_split(mk, nc, nbk, V, lda, W2, nb, bsplit, bsplit_elems, st);
            if (s) return s;
        }
    }
    bool prof = false;
    if (!partner) {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        prof = g_prof_on;
    }
    ProfRec rec{};
    if (prof) {
        HIP_TRY(hipEventCreate(&rec.a));
        HIP_TRY(hipEventCreate(&rec.b));
        HIP_TRY(hipEventRecord(rec.a, st));
    }
    ctqr_status s;
    if constexpr (sizeof(T) == 4) {
        if (bf16 == 2)
            s = gemm_nn_bf16x3(mk, nc, nbk, -1.0f, C, lda, bsplit, bsplit_elems, st, nullptr, partner ? 2 : 1);
        else
            s = gemm_nn<T>(mk, nc, nbk, V, lda, 1, W2, nb, T(-1), C, lda, nullptr, st, partner ? 0 : 1, 1, bf16);
    } else {
        (void)bsplit;
        (void)bsplit_elems;
        s = gemm_nn<T>(mk, nc, nbk, V, lda, 1, W2, nb, T(-1), C, lda, nullptr, st, partner ? 0 : 1, 1, 0);
    }
    if (s) return s;
    if (prof) {
        HIP_TRY(hipEventRecord(rec.b, st));
        rec.flops = 2.0 * (double)mk * (double)nc * (double)nbk;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof.push_back(rec);
    }
    return CTQR_OK;
}

// [G | W] = V^T B of one block column or pair (V: K x M Householder block,
// the first bmask columns of B too), into w.GW (column stride ldg).  Split
// BF16 splits V once for all the column tiles.
template <typename T>
ctqr_status block_reduction(int M, int N, int K, const T *V, int64_t lda, const T *B, int64_t ldb, int bmask,
                            FactorWS<T> &w, int ldg, int force_splits, hipStream_t st)
{
    bool prof = false;
    {
        std::lock_guard<std::mutex> lk(g_prof_mu);
        prof = g_prof_on;
    }
    ProfRec rec{};
    ctqr_status s = CTQR_OK;
    bool done = false;
    if constexpr (sizeof(T) == 4) {
        if (w.bf16 == 2) {
            if ((s = bf16x3_split_vt(K, M, V, lda, w.vtsplit, w.vtsplit_elems, st))) return s;
            if (prof) {
                HIP_TRY(hipEventCreate(&rec.a));
                HIP_TRY(hipEventCreate(&rec.b));
                HIP_TRY(hipEventRecord(rec.a, st));
            }
            // B's first bmask columns are V itself: G = V^T V, formed on and above its diagonal only
            s = gemm_tn_bf16x3(M, N, K, w.vtsplit, w.vtsplit_elems, B, ldb, bmask, 1.0f, 0.0f, w.GW, ldg, w.split,
                               SPLIT_PART_ELEMS, nullptr, st, force_splits, bmask);
            done = true;
        }
    }
    if (!done) {
        if (prof) {
            HIP_TRY(hipEventCreate(&rec.a));
            HIP_TRY(hipEventCreate(&rec.b));
            HIP_TRY(hipEventRecord(rec.a, st));
        }
        s = gemm_tn<T>(M, N, K, V, lda, M, B, ldb, bmask, T(1), T(0), w.GW, ldg, w.split, SPLIT_PART_ELEMS, nullptr,
                       st, force_splits, w.bf16);
    }
    if (s) return s;
    if (prof) {
        HIP_TRY(hipEventRecord(rec.b, st));
        rec.flops = 2.0 * (double)M * (double)N * (double)K;
        std::lock_guard<std::mutex> lk(g_prof_mu);
        g_prof_red.push_back(rec);
    }
    return CTQR_OK;
}

// Split counts of the two reductions of block k0 in the all-in-HBM
// factorization of an m x n matrix ([G | W] = V^T [V | C] and W' = T^T W).
// Every other caller that touches block k0's columns forces the same counts,
// so a column gets bit-identical updates whatever range it is processed in.
struct BlockSplits {
    int gw, tw;
};
BlockSplits block_splits(int m, int n, int nb, int k0)
{
    const int nbk = std::min(nb, n - k0), nc = n - (k0 + nbk);
    return {gemm_tn_splits(nbk, nbk + nc, m - k0), nc > 0 ? gemm_tn_splits(nbk, nc, nbk) : 1};
}

// The same for the group of block columns starting at kg: [G | W] over the
// group, then T_j^T (W_j - G_{j,<j} W'_{<j}) for each block j of the group.
struct GroupSplits {
    int gw;
    int t[GROUP];
};
GroupSplits group_splits(int m, int n, int nb, int kg)
{
    const int nbg = std::min(group_blocks(nb) * nb, n - kg), nc = n - (kg + nbg);
    GroupSplits s{};
    s.gw = gemm_tn_splits(nbg, nbg + std::max(nc, 0), m - kg);
    for (int j = 0; j * nb < nbg; ++j) {
        const int wj = std::min(nb, nbg - j * nb);
        s.t[j] = nc > 0 ? gemm_tn_splits(wj, nc, wj) : 1;
    }
    return s;
}

// Compact-WY update of nc columns C (rows from kg) by the group of block
// columns at kg (nbg Householder vectors Vg with Gram G = Vg^T Vg in Gs,
// column stride ldg).  With W = Vg^T C in Wg (column stride ldg), the rows of
// W' = T^T W for the group's factor T = [T_0, -T_0 G_01 T_1, ...; 0, T_1, ...]
// are, block by block, W'_j = T_j^T (W_j - G_{j,<j} W'_{<j}); then C -= Vg W'.
// G_{j,<j} is read as the transpose of G_{<j,j} (G is symmetric and only its
// diagonal and upper blocks are formed), unsplit so that every column range
// sums the same products in the same order.
template <typename T>
ctqr_status group_update(int m, int nb, int kg, int nbg, int nc, const T *Vg, int64_t lda, const T *Tf,
                         const T *Gs, T *Wg, int ldg, T *C, const GroupSplits &sp, FactorWS<T> &w, hipStream_t st)
{
    ctqr_status s;
    for (int j = 0, r0 = 0; r0 < nbg; ++j, r0 += nb) {
        const int wj = std::min(nb, nbg - r0);
        if (r0 > 0) {
            s = gemm_tn<T>(wj, nc, r0, Gs + (int64_t)r0 * ldg, ldg, 0, w.W2, ldg, 0, T(-1), T(1), Wg + r0, ldg, w.split,
                           SPLIT_PART_ELEMS, nullptr, st, 1);
            if (s) return s;
        }
        s = gemm_tn<T>(wj, nc, wj, Tf + (int64_t)(kg + r0) * nb, nb, 0, Wg + r0, ldg, 0, T(1), T(0), w.W2 + r0, ldg,
                       w.split, SPLIT_PART_ELEMS, nullptr, st, sp.t[j]);
        if (s) return s;
    }
    return trailing_update<T>(m - kg, nc, nbg, Vg, lda, w.W2, ldg, C, st, w.bf16, w.bsplit, w.bsplit_elems);
}

// Right-looking blocked Householder QR of the block columns [kb, ke) of an
// m x n matrix whose columns [kb, ce) are addressable through A (column k at
// A + k lda; ke <= ce), with every trailing update restricted to columns
// < ce.  kb, ke: multiples of nb (ke may be n).  With kb = 0, ke = ce = n it
// is the whole factorization.
template <typename T>
ctqr_status factor_blocks(int m, int n, T *A, int64_t lda, int nb, int kb, int ke, int ce, T *Tout, double *tau,
                          FactorWS<T> &w, unsigned *bars, ctqr_info *info, int ncu, hipStream_t st)
{
    ctqr_status s;
    for (int k0 = kb; k0 < ke; k0 += nb) {
        const int nbk = std::min(nb, n - k0);
        const BlockSplits sp = block_splits(m, n, nb, k0);
        // inner panels of the block column, each followed by its update of
        // the rest of the block column
        for (int c0 = k0; c0 < k0 + nbk; c0 += PANEL_W) {
            const int wdt = std::min(PANEL_W, k0 + nbk - c0);
            {
                PhaseScope ph(CTQR_PHASE_PANEL, st);
                // the panel's T is needed by the update of the rest of its block column
                s = panel_qr<T>(A, lda, m, c0, wdt, tau + c0, w.part, w.part2, w.gram_part, w.gram, w.Tin,
                                k0 + nbk - (c0 + wdt) > 0, bars + (int64_t)(c0 / PANEL_W) * GB_WORDS, info, ncu,
                                st);
                if (s) return s;
            }
            const int ncr = k0 + nbk - (c0 + wdt);
            if (ncr <= 0) continue;
            PhaseScope ph(CTQR_PHASE_INNER, st);
            const T *Vp = A + (int64_t)c0 * lda + c0;
            T *Cp = A + (int64_t)(c0 + wdt) * lda + c0;
            // W2 = T^T (V^T C): the split-K sum and the product with T^T in one launch
            s = gemm_tn_tprod<T>(wdt, ncr, m - c0, Vp, lda, wdt, Cp, lda, w.Tin, PANEL_W, w.GW, PANEL_W, w.W2,
                                 PANEL_W, w.split, SPLIT_PART_ELEMS, st);
            if (s) return s;
            // C -= V W' (rank 32) on 128 x 32 tiles: no columns padded to 128
            const int narrow_saved = gemm_narrow_max();
            gemm_set_narrow_max(std::max(narrow_saved, ncr));
            s = gemm_nn<T>(m - c0, ncr, wdt, Vp, lda, 1, w.W2, PANEL_W, T(-1), Cp, lda, nullptr, st);
            gemm_set_narrow_max(narrow_saved);
            if (s) return s;
        }
        const T *V = A + (int64_t)k0 * lda + k0;
        T *Tk = Tout + (int64_t)k0 * nb;
        const int g = group_blocks(nb), bi = (k0 / nb) % g, kg = k0 - bi * nb, ge = std::min(n, kg + g * nb);
        if (g > 1 && k0 + nbk < ge) {
            // not the last block of its group: its reflector updates the rest
            // of the group only
            if (kg < kb || ge > ke) return CTQR_EINVAL;   // ranges hold whole groups
            const int nr = ge - (k0 + nbk);
            {
                PhaseScope ph(CTQR_PHASE_REDUCTION, st);
                s = block_reduction<T>(nbk, nbk + nr, m - k0, V, lda, V, lda, nbk, w, nb,
                                       gemm_tn_splits(nbk, nbk + nr, m - k0), st);
                if (s) return s;
                if ((s = tbuild<T, T>(nbk, w.GW, nb, tau + k0, Tk, nb, w.Tw, st))) return s;
                s = gemm_tn<T>(nbk, nr, nbk, Tk, nb, 0, w.GW + (int64_t)nbk * nb, nb, 0, T(1), T(0), w.W2, nb,
                               w.split, SPLIT_PART_ELEMS, nullptr, st, gemm_tn_splits(nbk, nr, nbk));
                if (s) return s;
            }
            PhaseScope ph(CTQR_PHASE_GROUP_UPDATE, st);
            if ((s = trailing_update<T>(m - k0, nr, nbk, V, lda, w.W2, nb, A + (int64_t)(k0 + nbk) * lda + k0, st,
                                        w.bf16, w.bsplit, w.bsplit_elems, true)))
                return s;
            continue;
        }
        if (g > 1 && bi > 0) {
            // last block of a group: [G | W] = Vg^T [Vg | C] over the group,
            // this block's T from the Gram's diagonal block, then the group's
            // update of the rest
            const int nbg = ge - kg, ldg = g * nb;
            if (kg < kb) return CTQR_EINVAL;   // ranges hold whole groups
            const int nc = std::max(0, ce - ge);
            const GroupSplits gs = group_splits(m, n, nb, kg);
            const T *Vg = A + (int64_t)kg * lda + kg;
            {
                PhaseScope ph(CTQR_PHASE_REDUCTION, st);
                s = block_reduction<T>(nbg, nbg + nc, m - kg, Vg, lda, Vg, lda, nbg, w, ldg, gs.gw, st);
                if (s) return s;
                if ((s = tbuild<T, T>(nbk, w.GW + (int64_t)(bi * nb) * ldg + bi * nb, ldg, tau + k0, Tk, nb, w.Tw,
                                      st)))
                    return s;
            }
            // the Gram is kept for every group with columns to its right, also
            // those beyond this range (applied to them later)
            T *Gs = w.gstore + (int64_t)(kg / ldg) * ldg * ldg;
            if (ge < n)
                HIP_TRY(hipMemcpyAsync(Gs, w.GW, (size_t)ldg * nbg * sizeof(T), hipMemcpyDeviceToDevice, st));
            if (nc <= 0) continue;
            PhaseScope ph(CTQR_PHASE_UPDATE, st);
            if ((s = group_update<T>(m, nb, kg, nbg, nc, Vg, lda, Tout, Gs, w.GW + (int64_t)nbg * ldg, ldg,
                                     A + (int64_t)ge * lda + kg, gs, w, st)))
                return s;
            continue;
        }
        // block reflector of the whole block column: [G | W] = V^T [V | C]
        const int nc = std::max(0, ce - (k0 + nbk));
        {
            PhaseScope ph(CTQR_PHASE_REDUCTION, st);
            s = block_reduction<T>(nbk, nbk + nc, m - k0, V, lda, V, lda, nbk, w, nb, sp.gw, st);
            if (s) return s;
            if ((s = tbuild<T, T>(nbk, w.GW, nb, tau + k0, Tk, nb, w.Tw, st))) return s;
        }
        if (nc <= 0) continue;
        PhaseScope ph(CTQR_PHASE_UPDATE, st);
        // W' = T^T W;  C -= V W'
        s = gemm_tn<T>(nbk, nc, nbk, Tk, nb, 0, w.GW + (int64_t)nbk * nb, nb, 0, T(1), T(0), w.W2, nb,
                       w.split, SPLIT_PART_ELEMS, nullptr, st, sp.tw);
        if (s) return s;
        if ((s = trailing_update<T>(m - k0, nc, nbk, V, lda, w.W2, nb, A + (int64_t)(k0 + nbk) * lda + k0, st,
                                    w.bf16, w.bsplit, w.bsplit_elems)))
            return s;
    }
    return CTQR_OK;
}

// Left-looking application of the factored block columns [kb, ke) (their
// Householder blocks read through V: column k at V + k lda) to the columns
// [c0, c1) addressed through C (column k at C + k lda): for each block in
// order, W = V_k^T C, W' = T_k^T W, C -= V_k W', with the reductions split as
// in the all-in-HBM factorization.
template <typename T>
ctqr_status apply_blocks(int m, int n, const T *V, int64_t lda, const T *Tf, int nb, int kb, int ke, T *C, int c0,
                         int c1, FactorWS<T> &w, hipStream_t st)
{
    ctqr_status s;
    const int nc = c1 - c0;
    if (nc <= 0) return CTQR_OK;
    const int g = group_blocks(nb);
    for (int k0 = kb; k0 < ke; k0 += nb) {
        const int nbk = std::min(nb, n - k0);
        const T *Vk = V + (int64_t)k0 * lda + k0;
        T *Ck = C + (int64_t)c0 * lda + k0;
        if (g > 1 && k0 + nb < n) {
            // a group of two or more blocks, as the in-range update applies it
            const int nbg = std::min(g * nb, n - k0), ldg = g * nb;
            if ((k0 / nb) % g != 0 || k0 + nbg > ke) return CTQR_EINVAL;   // ranges hold whole groups
            const GroupSplits gs = group_splits(m, n, nb, k0);
            s = block_reduction<T>(nbg, nc, m - k0, Vk, lda, Ck, lda, 0, w, ldg, gs.gw, st);
            if (s) return s;
            if ((s = group_update<T>(m, nb, k0, nbg, nc, Vk, lda, Tf, w.gstore + (int64_t)(k0 / ldg) * ldg * ldg,
                                     w.GW, ldg, Ck, gs, w, st)))
                return s;
            k0 += nbg - nb;
            continue;
        }
        const BlockSplits sp = block_splits(m, n, nb, k0);
        // the in-HBM call forms [G | W] at once: its split count applies
        s = block_reduction<T>(nbk, nc, m - k0, Vk, lda, Ck, lda, 0, w, nb, sp.gw, st);
        if (s) return s;
        s = gemm_tn<T>(nbk, nc, nbk, Tf + (int64_t)k0 * nb, nb, 0, w.GW, nb, 0, T(1), T(0), w.W2, nb, w.split,
                       SPLIT_PART_ELEMS, nullptr, st, sp.tw);
        if (s) return s;
        if ((s = trailing_update<T>(m - k0, nc, nbk, Vk, lda, w.W2, nb, Ck, st, w.bf16, w.bsplit, w.bsplit_elems)))
            return s;
    }
    return CTQR_OK;
}

template <typename T>
ctqr_status factor_impl(int64_t m64, int64_t n64, T *A, int64_t lda, int nb, T *Tout, double *tau, T *Rinv,
                        void *work, ctqr_info *info, hipStream_t st, int bf16)
{
    const int m = (int)m64, n = (int)n64;
    FactorWS<T> w = carve_factor<T>(work, m64, n64, nb);
    w.bf16 = bf16;
    const int ncu = std::min(device_cus(), MAX_PANEL_WG);
    ctqr_status s;
    if ((s = info_reset(info, st))) return s;
    if ((s = fill_u32(w.bars, (ceil_div(n, PANEL_W) + 1) * GB_WORDS, 0u, st))) return s;
    if ((s = factor_blocks<T>(m, n, A, lda, nb, 0, n, n, Tout, tau, w, w.bars, info, ncu, st))) return s;
    PhaseScope ph(CTQR_PHASE_RINV, st);
    if ((s = rdiag_check<T>(n, A, lda, nullptr, info, st))) return s;
    return Rinv ? trinv_blocks<T>(n, A, lda, Rinv, w.rtmp, info, st) : CTQR_OK;
}

// Outer block width by timing: each candidate factors the leading columns of
// A (a multiple of every candidate, with the trailing updates over all n
// columns) and the fastest per factored column wins.  A is overwritten.
constexpr int TUNE_NB[3] = {64, 128, 256};
constexpr int TUNE_COLS = 1024;

template <typename T>
ctqr_status tune_nb_impl(int64_t m64, int64_t n64, T *A, int64_t lda, T *Tout, double *tau, void *work,
                         ctqr_info *info, hipStream_t st, int bf16, int32_t *nb_best, float *ms_per_col)
{
    const int m = (int)m64, n = (int)n64;
    // whole groups of block columns for every candidate (TUNE_COLS is a
    // multiple of each candidate's group width), or all n columns
    const int cols = std::min(n, TUNE_COLS);
    const int ncu = std::min(device_cus(), MAX_PANEL_WG);
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ctqr_status s = CTQR_OK;
    float best = 0.0f;
    int best_nb = TUNE_NB[2];
    HIP_TRY(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) {
        (void)hipEventDestroy(e0);
        return CTQR_EHIP;
    }
    for (int i = 0; i < 3 && !s; ++i) {
        const int nb = TUNE_NB[i];
        FactorWS<T> w = carve_factor<T>(work, m64, n64, nb);
        w.bf16 = bf16;
        if ((s = info_reset(info, st))) break;
        if ((s = fill_u32(w.bars, (ceil_div(n, PANEL_W) + 1) * GB_WORDS, 0u, st))) break;
        if (hipEventRecord(e0, st) != hipSuccess) { s = CTQR_EHIP; break; }
        if ((s = factor_blocks<T>(m, n, A, lda, nb, 0, cols, n, Tout, tau, w, w.bars, info, ncu, st))) break;
        float ms = 0.0f;
        if (hipEventRecord(e1, st) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
            hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
            s = CTQR_EHIP;
            break;
        }
        const float per = ms / (float)cols;
        if (ms_per_col) ms_per_col[i] = per;
        if (i == 0 || per < best) {
            best = per;
            best_nb = nb;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!s) *nb_best = best_nb;
    return s;
}

// ---------------------------------------------------------------------------
// Out-of-core factorization (Section II-B): the leading n_dev columns stay in
// HBM, the rest lives in pinned host memory and passes through HBM one tile of
// columns at a time.  The resident columns are factored right-looking with
// their trailing updates kept inside them; each host tile is then uploaded,
// takes the updates of every factored block to its left (left-looking: the
// resident blocks, then the earlier host tiles re-uploaded one by one), is
// factored, and is written back.  Every reduction uses the split count of
// the all-in-HBM factorization, so the factor is bit-identical to it.
// ---------------------------------------------------------------------------
template <typename T>
T *shift_cols(T *base, int64_t c0, int64_t lda)
{
    // column k of the returned pointer is column k - c0 of base (only
    // columns >= c0 are ever addressed through it)
    return reinterpret_cast<T *>(reinterpret_cast<uintptr_t>(base) - (uintptr_t)(c0 * lda * (int64_t)sizeof(T)));
}

template <typename T>
struct OocWS {
    FactorWS<T> f;
    T *D, *E, *diag;
    size_t bytes;
};

template <typename T>
OocWS<T> carve_ooc(void *work, int64_t m, int64_t n, int nb, int64_t lda, int64_t tile_cols)
{
    OocWS<T> o{};
    o.f = carve_factor<T>(work, m, n, nb);
    Carve c(work);
    c.off = o.f.bytes;
    o.D = c.take<T>(lda * tile_cols);
    o.E = c.take<T>(lda * tile_cols);
    o.diag = c.take<T>(n);
    o.bytes = c.off + 256;
    return o;
}

// Events and the copy stream of one out-of-core call; the compute stream
// waits for the copy stream's last work before the call returns, so the
// caller sees one stream-ordered operation.
struct CopyLane {
    hipStream_t cs = nullptr;
    std::vector<hipEvent_t> evs;
    ~CopyLane()
    {
        for (auto e : evs) (void)hipEventDestroy(e);
        if (cs) (void)hipStreamDestroy(cs);
    }
    ctqr_status init()
    {
        HIP_TRY(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
        return CTQR_OK;
    }
    // records a fresh event on stream s
    ctqr_status mark(hipStream_t s, hipEvent_t *out)
    {
        hipEvent_t e;
        HIP_TRY(hipEventCreateWithFlags(&e, hipEventDisableTiming));
        evs.push_back(e);
        HIP_TRY(hipEventRecord(e, s));
        *out = e;
        return CTQR_OK;
    }
    ctqr_status wait(hipStream_t s, hipEvent_t e)
    {
        if (e) HIP_TRY(hipStreamWaitEvent(s, e, 0));
        return CTQR_OK;
    }
};

template <typename T>
ctqr_status factor_ooc_impl(int64_t m64, int64_t n64, T *A_dev, T *A_host, int64_t lda, int64_t n_dev64,
                            int64_t tile64, int nb, T *Tout, double *tau, T *Rinv, void *work, ctqr_info *info,
                            hipStream_t st, int bf16)
{
    const int m = (int)m64, n = (int)n64, n_dev = (int)n_dev64, tile = (int)tile64;
    OocWS<T> o = carve_ooc<T>(work, m64, n64, nb, lda, tile64);
    FactorWS<T> &w = o.f;
    w.bf16 = bf16;
    const int ncu = std::min(device_cus(), MAX_PANEL_WG);
    const size_t col_bytes = (size_t)lda * sizeof(T);
    auto host_cols = [&](int c0) { return A_host + (int64_t)(c0 - n_dev) * lda; };
    auto tile_bytes = [&](int c0) { return (size_t)(std::min(n, c0 + tile) - c0) * col_bytes; };
    ctqr_status s;
    if ((s = info_reset(info, st))) return s;
    if ((s = fill_u32(w.bars, (ceil_div(n, PANEL_W) + 1) * GB_WORDS, 0u, st))) return s;
    // Two tile buffers: X holds the tile being updated and factored, Y the
    // earlier tiles re-uploaded for their updates, then the next tile
    // (prefetched while X is factored); they swap roles every tile.  All
    // copies go through the copy stream.
    CopyLane cl;
    if ((s = cl.init())) return s;
    T *buf[2] = {o.D, o.E};
    int x = 0;
    hipEvent_t loaded_x = nullptr, free_y = nullptr, last_copy = nullptr;
    if (n_dev < n) {   // the first host tile streams in while the resident columns are factored
        HIP_TRY(hipMemcpyAsync(buf[x], host_cols(n_dev), tile_bytes(n_dev), hipMemcpyHostToDevice, cl.cs));
        if ((s = cl.mark(cl.cs, &loaded_x))) return s;
        last_copy = loaded_x;
    }
    if (n_dev > 0) {
        // in pieces of 8192 columns (the same arithmetic as one call), each
        // followed by a progress mark
        for (int k0 = 0; k0 < n_dev; k0 += 8192) {
            const int k1 = std::min(n_dev, k0 + 8192);
            if ((s = factor_blocks<T>(m, n, A_dev, lda, nb, k0, k1, n_dev, Tout, tau, w, w.bars, info, ncu, st)))
                return s;
            if ((s = progress_mark(st, CTQR_PROGRESS_FACTOR, k1, n))) return s;
        }
        if ((s = diag_copy<T>(0, n_dev, A_dev, lda, o.diag, st))) return s;
        if (Rinv && (s = trinv_blocks_range<T>(n, 0, n_dev, A_dev, lda, Rinv, w.rtmp, st))) return s;
    }
    for (int c0 = n_dev; c0 < n; c0 += tile) {
        const int c1 = std::min(n, c0 + tile);
        const int y = x ^ 1;
        if ((s = cl.wait(st, loaded_x))) return s;
        T *Dv = shift_cols(buf[x], c0, lda);
        if (n_dev > 0 && (s = apply_blocks<T>(m, n, A_dev, lda, Tout, nb, 0, n_dev, Dv, c0, c1, w, st))) return s;
        for (int e0 = n_dev; e0 < c0; e0 += tile) {
            const int e1 = std::min(n, e0 + tile);
            if ((s = cl.wait(cl.cs, free_y))) return s;
            HIP_TRY(hipMemcpyAsync(buf[y], host_cols(e0), tile_bytes(e0), hipMemcpyHostToDevice, cl.cs));
            hipEvent_t ready;
            if ((s = cl.mark(cl.cs, &ready))) return s;
            last_copy = ready;
            if ((s = cl.wait(st, ready))) return s;
            T *Ev = shift_cols(buf[y], e0, lda);
            if ((s = apply_blocks<T>(m, n, Ev, lda, Tout, nb, e0, e1, Dv, c0, c1, w, st))) return s;
            if ((s = cl.mark(st, &free_y))) return s;
        }
        if ((s = factor_blocks<T>(m, n, Dv, lda, nb, c0, c1, c1, Tout, tau, w, w.bars, info, ncu, st))) return s;
        if ((s = diag_copy<T>(c0, c1, Dv, lda, o.diag, st))) return s;
        if (Rinv && (s = trinv_blocks_range<T>(n, c0, c1, Dv, lda, Rinv, w.rtmp, st))) return s;
        hipEvent_t factored;
        if ((s = cl.mark(st, &factored))) return s;
        if ((s = progress_mark(st, CTQR_PROGRESS_FACTOR, c1, n))) return s;
        // next tile into Y (after Y's last update read), then this tile back
        hipEvent_t loaded_next = nullptr;
        if (c1 < n) {
            if ((s = cl.wait(cl.cs, free_y))) return s;
            HIP_TRY(hipMemcpyAsync(buf[y], host_cols(c1), tile_bytes(c1), hipMemcpyHostToDevice, cl.cs));
            if ((s = cl.mark(cl.cs, &loaded_next))) return s;
        }
        if ((s = cl.wait(cl.cs, factored))) return s;
        HIP_TRY(hipMemcpyAsync(host_cols(c0), buf[x], (size_t)(c1 - c0) * col_bytes, hipMemcpyDeviceToHost, cl.cs));
        hipEvent_t written;
        if ((s = cl.mark(cl.cs, &written))) return s;
        last_copy = written;
        // swap: the written-back buffer takes the re-uploads of the next tile
        x = y;
        loaded_x = loaded_next;
        free_y = written;
    }
    if ((s = cl.wait(st, last_copy))) return s;
    // rank check over the diagonal collected above (stride 0: diag[k])
    if ((s = rdiag_check<T>(n, o.diag, 0, nullptr, info, st))) return s;
    // the copy stream and its events are released only once idle
    HIP_TRY(hipStreamSynchronize(cl.cs));
    return CTQR_OK;
}

// Sets the slice-tile choice of the GEMMs enqueued by this thread for the
// lifetime of the scope.
struct NarrowScope {
    int old;
    explicit NarrowScope(int v) : old(gemm_narrow_max()) { gemm_set_narrow_max(v); }
    ~NarrowScope() { gemm_set_narrow_max(old); }
};

constexpr int DEFAULT_NARROW = 32;   // slices up to which the 32-wide tile is used

// One multi-slice solve over a carved workspace, in three phases: the first
// two enqueue no host synchronisation when host_sync is off, so a graph can
// capture them.
template <typename T>
struct SolveRun {
    int m, n, nb, S;
    const T *QR;
    int64_t lda;
    const T *Tf;
    const T *Rinv;   // the factor's diagonal-block inverses, or null (built into w.Rinv)
    const double *B;
    int64_t ldb;
    const ctqr_sparse *A64;
    double tol;
    int max_iters;
    int method;      // CTQR_REFINE_CSNE or CTQR_REFINE_PCG
    bool progress;   // report each refinement iteration to the progress hook
    bool pageable;   // read the end-of-refinement flag into ordinary host memory (no pinned word)
    int narrow;
    ctqr_info *info;
    SolveWS<T> w;
    int64_t sp_elems;
    TrsmParts tp{};  // split-BF16 parts of the refinement's substitutions (tp.x null: none)
    bool split_r;    // R's parts are made by this run, not kept by a solver
    bool rparts_made = false;   // ... and already made (before the first substitution)
    bool fused;      // Q^T B and the substitutions as the persistent kernels (few slices, factor in HBM)
    bool refine() const { return A64 != nullptr && max_iters > 0; }
    const TrsmParts *parts() const { return tp.x ? &tp : nullptr; }
};

// The persistent kernels take at most FUSED_MAX_S slices, block reflectors
// of whole 64-row chunks up to 256 wide, and right-hand sides whose rows fit
// their LDS.  They are selected by the environment variable CTQR_FUSED=1,
// read at every solve: on MI355X the launch-per-block chains are faster at
// every slice count measured (each compute unit owns too few rows of R for
// long column reads), so they are the default.
bool fused_enabled()
{
    const char *e = std::getenv("CTQR_FUSED");
    return e && e[0] == '1';
}

template <typename T>
bool fused_eligible(int64_t m, int nb, int S)
{
    return fused_enabled() && S <= FUSED_MAX_S && nb % 64 == 0 && nb <= 256 && fused_fits(m, sizeof(T));
}

template <typename T>
SolveRun<T> make_run(int64_t m, int64_t n, const T *QR, int64_t lda, const T *Tf, const T *Rinv, int nb,
                     const double *B, int64_t ldb, int S, const ctqr_sparse *A64, double tol, int max_iters,
                     void *work, ctqr_info *info, bool carve_rinv, int method = CTQR_REFINE_CSNE,
                     int trsm_split = TRSM_PARTS_NONE)
{
    SolveRun<T> r{};
    r.m = (int)m; r.n = (int)n; r.nb = nb; r.S = S;
    r.QR = QR; r.lda = lda; r.Tf = Tf; r.Rinv = Rinv; r.B = B; r.ldb = ldb;
    r.A64 = A64; r.tol = tol; r.max_iters = max_iters; r.method = method;
    r.narrow = S <= DEFAULT_NARROW ? DEFAULT_NARROW : 0;
    r.info = info;
    r.w = carve_solve<T>(work, m, n, nb, S, r.refine() ? (method == CTQR_REFINE_PCG ? 2 : 1) : 0, carve_rinv,
                         trsm_split);
    r.sp_elems = std::max<int64_t>(SPLIT_PART_ELEMS, 64LL * nb * S);
    r.tp.x = r.w.xparts;
    r.tp.r = r.w.rparts;
    r.split_r = r.w.rparts != nullptr;
    r.fused = fused_eligible<T>(m, nb, S) && r.w.fex != nullptr;
    return r;
}

// Q^T B over the block reflectors [kb, ke) (Householder blocks read through
// V: column k at V + k lda), one block at a time: B -= V (T^T (V^T B)).
template <typename T>
ctqr_status apply_qt_range(SolveRun<T> &r, const T *QRv, int kb, int ke, hipStream_t st)
{
    SolveWS<T> &w = r.w;
    const int m = r.m, n = r.n, nb = r.nb, S = r.S;
    ctqr_status s;
    for (int k0 = kb; k0 < ke; k0 += nb) {
        const int nbk = std::min(nb, n - k0);
        const T *V = QRv + (int64_t)k0 * r.lda + k0;
        T *Bk = w.Bw + k0;
        s = gemm_tn<T>(nbk, S, m - k0, V, r.lda, nbk, Bk, w.ldbw, 0, T(1), T(0), w.W, nb, w.split, r.sp_elems,
                       nullptr, st);
        if (s) return s;
        s = gemm_tn<T>(nbk, S, nbk, r.Tf + (int64_t)k0 * nb, nb, 0, w.W, nb, 0, T(1), T(0), w.W2, nb, w.split,
                       r.sp_elems, nullptr, st);
        if (s) return s;
        if constexpr (sizeof(T) == 4) {
            if (w.qsplit) {
                // refined solve of many slices: B_k -= V W' on split-BF16 MFMA
                // (the refinement's corrections need the factor's accuracy only)
                s = bf16x3_split(m - k0, S, nbk, V, r.lda, w.W2, nb, w.qsplit, w.qsplit_elems, st);
                if (!s) s = gemm_nn_bf16x3(m - k0, S, nbk, -1.0f, Bk, w.ldbw, w.qsplit, w.qsplit_elems, st, nullptr, 2);
                if (s) return s;
                continue;
            }
        }
        s = gemm_nn<T>(m - k0, S, nbk, V, r.lda, 1, w.W2, nb, T(-1), Bk, w.ldbw, nullptr, st);
        if (s) return s;
    }
    return CTQR_OK;
}

// Clears the refinement's history, norms and (conjugate-gradient form) the
// search direction and per-slice scalars.
template <typename T>
ctqr_status refine_setup(SolveRun<T> &r, hipStream_t st)
{
    SolveWS<T> &w = r.w;
    const int S = r.S;
    ctqr_status s;
    if ((s = fill_f64(w.hist, 8, 0.0, st))) return s;
    if ((s = fill_u32((unsigned *)w.dmax, 2LL * S, 0u, st))) return s;
    if ((s = fill_u32((unsigned *)w.xmax, 2LL * S, 0u, st))) return s;
    if ((s = fill_u32((unsigned *)w.smax, 2LL * S, 0u, st))) return s;
    if constexpr (sizeof(T) == 4) {
        if (r.split_r && !r.rparts_made && (s = trsm_split_r(r.n, r.QR, r.lda, w.rparts, st))) return s;
        r.rparts_made = r.split_r;
    }
    if (r.method != CTQR_REFINE_PCG) return CTQR_OK;
    if ((s = fill_f64(w.p, (int64_t)r.n * S, 0.0, st))) return s;
    return fill_f64(w.gamma, S, 0.0, st);
}

// Q^T B and the back substitution (Section II-C), then the set-up of the
// refinement.
template <typename T>
ctqr_status solve_start(SolveRun<T> &r, hipStream_t st)
{
    NarrowScope ns(r.narrow);
    SolveWS<T> &w = r.w;
    const int m = r.m, n = r.n, nb = r.nb, S = r.S;
    ctqr_status s;
    if ((s = info_reset(r.info, st))) return s;
    if ((s = fill_u32((unsigned *)w.done, 64, 0u, st))) return s;
    {
        // working copy of B in the factor's precision
        PhaseScope ph(CTQR_PHASE_QTB, st);
        if (r.fused) {
            s = qtb_fused<T>(m, n, nb, S, r.QR, r.lda, r.Tf, r.B, r.ldb, w.Bw, w.ldbw, w.fex, w.fbar, r.info, st);
            if (s) return s;
        } else {
            if ((s = copy_cm<T, double>(m, S, r.B, r.ldb, w.Bw, w.ldbw, st))) return s;
            if ((s = apply_qt_range(r, r.QR, 0, n, st))) return s;
        }
    }
    {
        // back substitution R X = (Q^T B)[0:n], with the factor's diagonal-block
        // inverses (built here when the factor was stored without them)
        PhaseScope ph(CTQR_PHASE_TRSM, st);
        if (!r.Rinv) {
            if ((s = trinv_blocks<T>(n, r.QR, r.lda, w.Rinv, w.RinvT, r.info, st))) return s;
            r.Rinv = w.Rinv;
        }
        // A solution that the refinement corrects needs the factor's own
        // accuracy only, as the refinement's substitutions do: with R's
        // split-BF16 parts (made here once for the run) the off-diagonal
        // products take them too.
        const TrsmParts *rp = nullptr;
        if constexpr (sizeof(T) == 4) {
            if (r.refine() && r.split_r && !r.rparts_made) {
                if ((s = trsm_split_r(r.n, r.QR, r.lda, w.rparts, st))) return s;
                r.rparts_made = true;
            }
            if (r.refine()) rp = r.parts();
        }
        if (r.fused)
            s = trsm_fused<T>(n, S, false, r.QR, r.lda, r.Rinv, w.Bw, w.ldbw, w.Xw, w.ldxw, w.fex, w.fbar, nullptr,
                              r.info, st);
        else
            s = trsm_upper<T>(n, S, r.QR, r.lda, r.Rinv, w.Bw, w.ldbw, w.Xw, w.ldxw, w.split, r.sp_elems, nullptr,
                              st, rp);
        if (s) return s;
    }
    PhaseScope ph(CTQR_PHASE_REFINE_OTHER, st);
    if (!r.refine()) return CTQR_OK;
    if ((s = cm_to_rm<double, T>(n, S, w.Xw, w.ldxw, w.xr, nullptr, st))) return s;
    if ((s = cm_to_rm<double, double>(m, S, r.B, r.ldb, w.Br, nullptr, st))) return s;
    return refine_setup(r, st);
}

// Reads the device-side end-of-refinement flag (synchronises the stream).
ctqr_status read_done(const int *done, hipStream_t st, bool &out, bool pageable = false)
{
    if (pageable) {
        int v = 0;
        HIP_TRY(hipMemcpyAsync(&v, done, sizeof(int), hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        out = v != 0;
        return CTQR_OK;
    }
    int *flag = host_flag();
    if (!flag) return CTQR_EHIP;
    HIP_TRY(hipMemcpyAsync(flag, done, sizeof(int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
    out = *flag != 0;
    return CTQR_OK;
}

// Refinement iterations it0 .. it1-1 with FP64 residuals against the sparse A
// (r = B - A x, s = A^T r) and the preconditioner (R^T R)^-1, applied by
// minv (s32 -> d32 through y32: R^T y = s, R d = y, in the factor's
// precision).  CTQR_REFINE_CSNE adds the correction, x += d (corrected
// semi-normal equations); CTQR_REFINE_PCG combines the corrections as
// conjugate directions (refine.hip).  Every kernel of an iteration returns at
// once after the device-side flag has ended the refinement.  With host_sync
// the loop stops enqueuing once that flag is set; *ran is then the number of
// iterations the refinement took.
template <typename T, typename MInv>
ctqr_status refine_iters_with(SolveRun<T> &r, int it0, int it1, bool host_sync, hipStream_t st, int *ran, MInv minv)
{
    NarrowScope ns(r.narrow);
    SolveWS<T> &w = r.w;
    const int m = r.m, n = r.n, S = r.S;
    const ctqr_sparse *A = r.A64;
    const bool pcg = r.method == CTQR_REFINE_PCG;
    ctqr_status s;
    if (ran) *ran = it1;
    for (int it = it0; it < it1; ++it) {
        const int *skip = w.done;
        {
            PhaseScope ph(CTQR_PHASE_RESIDUAL, st);
            s = spmm_rowmajor(m, S, A->rowptr, A->col, A->val, -1.0, w.xr, 1.0, w.Br, w.r, skip, st);
            if (s) return s;
            s = spmm_rowmajor(n, S, A->colptr, A->row, A->cval, 1.0, w.r, 0.0, nullptr, w.s, skip, st,
                              pixel_tile_side(n));
            if (s) return s;
            if ((s = slice_absmax(n, S, w.s, w.smax, skip, st))) return s;
        }
        {
            PhaseScope ph(CTQR_PHASE_REFINE_TRSM, st);
            if ((s = rm_to_cm<T, double>(n, S, w.s, w.s32, w.ldxw, skip, st))) return s;
            if ((s = minv(skip))) return s;
        }
        PhaseScope ph(CTQR_PHASE_REFINE_OTHER, st);
        if (!pcg) {
            if ((s = refine_update<T>(n, S, w.xr, w.d32, w.ldxw, w.dmax, w.xmax, w.xs, skip, st))) return s;
        } else {
            double *z = (it & 1) ? w.z1 : w.z0, *zp = (it & 1) ? w.z0 : w.z1;
            if ((s = cm_to_rm<double, T>(n, S, w.d32, w.ldxw, z, skip, st))) return s;
            if ((s = slice_dot(n, S, w.s, z, w.dpart, w.sz, skip, st))) return s;
            if (it > 0 && (s = slice_dot(n, S, w.s, zp, w.dpart, w.szp, skip, st))) return s;
            if ((s = pcg_beta(S, it == 0, w.sz, w.szp, w.gamma, w.beta, skip, st))) return s;
            if ((s = pcg_direction(n, S, z, w.beta, w.p, skip, st))) return s;
            s = spmm_rowmajor(m, S, A->rowptr, A->col, A->val, 1.0, w.p, 0.0, nullptr, w.q, skip, st);
            if (s) return s;
            if ((s = slice_dot(m, S, w.q, w.q, w.dpart, w.qq, skip, st))) return s;
            if ((s = pcg_alpha(S, w.gamma, w.qq, w.alpha, skip, st))) return s;
            if ((s = pcg_step(n, S, w.xr, w.p, w.alpha, w.dmax, w.xmax, w.xs, skip, st))) return s;
        }
        // conjugate-gradient steps need not shrink monotonically: a longer
        // run of non-contracting steps ends that form
        s = refine_check(S, w.dmax, w.xmax, w.smax, w.s0, r.tol, it, r.max_iters, pcg ? 6 : 2, w.hist, w.done,
                         r.info, st);
        if (s) return s;
        if ((s = refine_keep((int64_t)n * S, w.xs, w.xbest, w.hist, st))) return s;
        if (r.progress && (s = progress_mark(st, CTQR_PROGRESS_SOLVE, it + 1, r.max_iters))) return s;
        if (host_sync) {
            bool done = false;
            if ((s = read_done(w.done, st, done, r.pageable))) return s;
            if (done) {
                if (ran) *ran = it + 1;
                break;
            }
        }
    }
    return CTQR_OK;
}

// In-HBM factor: the two block substitutions of trsm.hip
template <typename T>
ctqr_status refine_iters(SolveRun<T> &r, int it0, int it1, bool host_sync, hipStream_t st, int *ran)
{
    SolveWS<T> &w = r.w;
    auto minv = [&](const int *skip) -> ctqr_status {
        if (r.fused) {
            ctqr_status s = trsm_fused<T>(r.n, r.S, true, r.QR, r.lda, r.Rinv, w.s32, w.ldxw, w.y32, w.ldxw, w.fex,
                                          w.fbar, skip, r.info, st);
            if (s) return s;
            return trsm_fused<T>(r.n, r.S, false, r.QR, r.lda, r.Rinv, w.y32, w.ldxw, w.d32, w.ldxw, w.fex, w.fbar,
                                 skip, r.info, st);
        }
        ctqr_status s = trsm_upper_trans<T>(r.n, r.S, r.QR, r.lda, r.Rinv, w.s32, w.ldxw, w.y32, w.ldxw, w.split,
                                            r.sp_elems, skip, st, r.parts());
        if (s) return s;
        return trsm_upper<T>(r.n, r.S, r.QR, r.lda, r.Rinv, w.y32, w.ldxw, w.d32, w.ldxw, w.split, r.sp_elems, skip,
                             st, r.parts());
    };
    return refine_iters_with(r, it0, it1, host_sync, st, ran, minv);
}

// After the refinement: a refinement that did not converge returns the
// iterate with the smallest update after it (device-side decision).
template <typename T>
ctqr_status refine_finish(SolveRun<T> &r, hipStream_t st)
{
    if (!r.refine()) return CTQR_OK;
    return refine_select((int64_t)r.n * r.S, r.w.xr, r.w.xbest, r.w.hist, r.info, st);
}

// The first S_out slices of the solution into X (FP64, column-major).
template <typename T>
ctqr_status solve_finish(SolveRun<T> &r, int S_out, double *X, int64_t ldx, hipStream_t st)
{
    SolveWS<T> &w = r.w;
    if (!r.refine()) return copy_cm<double, T>(r.n, S_out, w.Xw, w.ldxw, X, ldx, st);
    ctqr_status s = refine_finish(r, st);
    if (s) return s;
    if (S_out == r.S) return rm_to_cm<double, double>(r.n, r.S, w.xr, X, ldx, nullptr, st);
    // row-major x holds S slices per row: gather the first S_out of each
    return rm_to_cm_sub(r.n, r.S, S_out, w.xr, X, ldx, st);
}

template <typename T>
ctqr_status solve_impl(int64_t m64, int64_t n64, const T *QR, int64_t lda, const T *Tf,
                       const double *tau, const T *Rinv_in, int nb, const double *B, int64_t ldb, int S,
                       double *X, int64_t ldx, const ctqr_sparse *A64, double tol, int max_iters, int method,
                       void *work, ctqr_info *info, hipStream_t st, bool pageable = false)
{
    (void)tau;
    SolveRun<T> r = make_run<T>(m64, n64, QR, lda, Tf, Rinv_in, nb, B, ldb, S, A64, tol, max_iters, work, info,
                                true, method, TRSM_PARTS_ALL);
    r.pageable = pageable;
    ctqr_status s = solve_start(r, st);
    if (s) return s;
    if (r.refine() && (s = refine_iters(r, 0, max_iters, true, st, nullptr))) return s;
    return solve_finish(r, S, X, ldx, st);
}

// ---------------------------------------------------------------------------
// Out-of-core solve: the factor of ctqr_qr_factor_ooc, resident columns in
// HBM and the rest in pinned host memory.  Q^T B takes the resident blocks,
// then each host tile uploaded in turn; R X = C runs right-looking from the
// last tile back to the resident part and R^T Y = C left-looking from the
// resident part forward, so every step reads only its own column block and
// every pass uploads each tile once.
// ---------------------------------------------------------------------------
template <typename T>
struct TileCache {
    const T *host;
    T *buf;
    int64_t lda;
    int n_dev, tile, n;
    int loaded = -1;   // first column of the tile the buffer holds
    // the tile starting at column c0, uploaded unless the buffer holds it;
    // returns the column-shifted pointer (column k at + k lda)
    ctqr_status get(int c0, hipStream_t st, const T **out)
    {
        if (loaded != c0) {
            const int c1 = std::min(n, c0 + tile);
            HIP_TRY(hipMemcpyAsync(buf, host + (int64_t)(c0 - n_dev) * lda, (size_t)(c1 - c0) * lda * sizeof(T),
                                   hipMemcpyHostToDevice, st));
            loaded = c0;
        }
        *out = shift_cols(buf, c0, lda);
        return CTQR_OK;
    }
};

template <typename T>
ctqr_status ooc_upper(SolveRun<T> &r, TileCache<T> &tc, const T *QRdev, T *C, int64_t ldc, T *X, int64_t ldx,
                      const int *skip, hipStream_t st)
{
    ctqr_status s;
    const int n = r.n;
    int last = tc.n_dev + (int)((n - tc.n_dev - 1) / tc.tile) * tc.tile;
    for (int c0 = last; c0 >= tc.n_dev && c0 < n; c0 -= tc.tile) {
        const T *Rv;
        if ((s = tc.get(c0, st, &Rv))) return s;
        s = trsm_upper_cols<T>(n, r.S, Rv, r.lda, r.Rinv, C, ldc, X, ldx, c0, std::min(n, c0 + tc.tile),
                               r.w.split, r.sp_elems, skip, st);
        if (s) return s;
    }
    if (tc.n_dev > 0)
        return trsm_upper_cols<T>(n, r.S, QRdev, r.lda, r.Rinv, C, ldc, X, ldx, 0, tc.n_dev, r.w.split,
                                  r.sp_elems, skip, st);
    return CTQR_OK;
}

template <typename T>
ctqr_status ooc_upper_trans(SolveRun<T> &r, TileCache<T> &tc, const T *QRdev, T *C, T *Y, const int *skip,
                            hipStream_t st)
{
    ctqr_status s;
    const int n = r.n;
    if (tc.n_dev > 0) {
        s = trsm_upper_trans_cols<T>(n, r.S, QRdev, r.lda, r.Rinv, C, r.w.ldxw, Y, r.w.ldxw, 0, tc.n_dev,
                                     r.w.split, r.sp_elems, skip, st);
        if (s) return s;
    }
    for (int c0 = tc.n_dev; c0 < n; c0 += tc.tile) {
        const T *Rv;
        if ((s = tc.get(c0, st, &Rv))) return s;
        s = trsm_upper_trans_cols<T>(n, r.S, Rv, r.lda, r.Rinv, C, r.w.ldxw, Y, r.w.ldxw, c0,
                                     std::min(n, c0 + tc.tile), r.w.split, r.sp_elems, skip, st);
        if (s) return s;
    }
    return CTQR_OK;
}

template <typename T>
ctqr_status solve_ooc_impl(int64_t m64, int64_t n64, const T *QR_dev, const T *QR_host, int64_t lda, int n_dev,
                           int tile, const T *Tf, const T *Rinv, int nb, const double *B, int64_t ldb, int S,
                           double *X, int64_t ldx, const ctqr_sparse *A64, double tol, int max_iters, int method,
                           void *work, ctqr_info *info, hipStream_t st)
{
    SolveRun<T> r = make_run<T>(m64, n64, QR_dev, lda, Tf, Rinv, nb, B, ldb, S, A64, tol, max_iters, work, info,
                                false, method);
    r.fused = false;   // the column tiles of the factor stream through; the persistent kernels need all of it
    r.progress = true;
    Carve c(work);
    c.off = r.w.bytes;
    TileCache<T> tc{QR_host, c.take<T>(lda * (int64_t)tile), lda, n_dev, tile, (int)n64};
    NarrowScope ns(r.narrow);
    SolveWS<T> &w = r.w;
    const int m = r.m, n = r.n;
    ctqr_status s;
    if ((s = info_reset(info, st))) return s;
    if ((s = fill_u32((unsigned *)w.done, 64, 0u, st))) return s;
    if ((s = copy_cm<T, double>(m, S, B, ldb, w.Bw, w.ldbw, st))) return s;
    if (n_dev > 0 && (s = apply_qt_range(r, QR_dev, 0, n_dev, st))) return s;
    for (int c0 = n_dev; c0 < n; c0 += tile) {
        const T *Vv;
        if ((s = tc.get(c0, st, &Vv))) return s;
        if ((s = apply_qt_range(r, Vv, c0, std::min(n, c0 + tile), st))) return s;
    }
    if ((s = progress_mark(st, CTQR_PROGRESS_SOLVE, 0, max_iters))) return s;
    // R X = (Q^T B)[0:n], substituting in the working copy
    if ((s = ooc_upper(r, tc, QR_dev, w.Bw, w.ldbw, w.Xw, w.ldxw, nullptr, st))) return s;
    if (!r.refine()) return copy_cm<double, T>(n, S, w.Xw, w.ldxw, X, ldx, st);
    if ((s = cm_to_rm<double, T>(n, S, w.Xw, w.ldxw, w.xr, nullptr, st))) return s;
    if ((s = cm_to_rm<double, double>(m, S, B, ldb, w.Br, nullptr, st))) return s;
    if ((s = refine_setup(r, st))) return s;
    auto minv = [&](const int *skip) -> ctqr_status {
        ctqr_status e = ooc_upper_trans(r, tc, QR_dev, w.s32, w.y32, skip, st);
        if (e) return e;
        return ooc_upper(r, tc, QR_dev, w.y32, w.ldxw, w.d32, w.ldxw, skip, st);
    };
    if ((s = refine_iters_with(r, 0, max_iters, true, st, nullptr, minv))) return s;
    if ((s = refine_finish(r, st))) return s;
    return rm_to_cm<double, double>(n, S, w.xr, X, ldx, nullptr, st);
}

// ---------------------------------------------------------------------------
// Batched solver: one stored factor serves a stream of requests (the
// factorization does not depend on B and is computed once, Section II-A; the
// per-slice cost falls as more slices share one read of the factor,
// Section III-B).  Requests are padded to a slice bucket (powers of two up to
// 64, multiples of 64 above); each bucket's solve is captured once into a HIP
// graph and replayed.
// ---------------------------------------------------------------------------
constexpr int SOLVER_MAX_SLICES = 4096;
constexpr int GRAPH_EXTRA_ITERS = 2;   // refinement iterations beyond the calibrated count

struct SolverBucket {
    int S = 0;
    int narrow = 0;            // slice-tile threshold of its GEMMs
    int iters = -1;            // refinement iterations of its calibration run (-1: none yet)
    int graph_iters = 0;       // refinement iterations the graph holds (or a direct run enqueues)
    hipGraphExec_t exec = nullptr;
    bool direct = false;       // run through the persistent kernels, without a graph
};

int next_pow2(int x)
{
    int p = 1;
    while (p < x) p <<= 1;
    return p;
}

// Slice buckets: powers of two up to 64, then multiples of 64 (a request is
// padded by less than 64 slices beyond 64).
constexpr int BUCKET_STEP = 64;
int bucket_cap(int max_slices)
{
    return max_slices <= BUCKET_STEP ? next_pow2(max_slices) : (int)round_up(max_slices, BUCKET_STEP);
}
std::vector<int> bucket_sizes(int cap)
{
    std::vector<int> v;
    for (int b = 1; b <= std::min(cap, BUCKET_STEP); b <<= 1) v.push_back(b);
    for (int b = 2 * BUCKET_STEP; b <= cap; b += BUCKET_STEP) v.push_back(b);
    return v;
}

}  // namespace

struct ctqr_solver_t {
    ctqr_solver_desc d{};
    ctqr_sparse sp{};
    bool refine = false;
    int smax = 0;
    int64_t ldbp = 0;
    double *Bpad = nullptr;     // m x smax request buffer the graphs read
    ctqr_info *info = nullptr;  // device info the graphs write
    void *swork = nullptr;      // solve workspace of the largest bucket
    __bf16 *rparts = nullptr;   // R's split-BF16 parts (wide refined buckets), made once
    bool rparts_ready = false;
    hipStream_t cap = nullptr;  // capture stream (never executes work)
    hipEvent_t last = nullptr;  // recorded after each call's work, waited for by the next call
    std::vector<SolverBucket> buckets;
    std::mutex mu;
};

// Calls on different streams share the request buffer and the workspace: each
// call's stream first waits for the work of the previous call, and records
// the end of its own.
struct SolverOrder {
    ctqr_solver_t *sv;
    hipStream_t st;
    ctqr_status begin()
    {
        HIP_TRY(hipStreamWaitEvent(st, sv->last, 0));
        return CTQR_OK;
    }
    ctqr_status end()
    {
        HIP_TRY(hipEventRecord(sv->last, st));
        return CTQR_OK;
    }
};

namespace {

struct SolverLayout {
    ctqr_info *info;
    double *Bpad;
    __bf16 *rparts;   // R's split-BF16 parts for the wide refined buckets, or null
    void *swork;
    size_t bytes;
};

SolverLayout solver_layout(const ctqr_solver_desc *d, void *work, int smax, int64_t ldbp)
{
    Carve c(work);
    SolverLayout L{};
    L.info = c.take<ctqr_info>(1);
    L.Bpad = c.take<double>(ldbp * smax);
    const int refine = d->A64 != nullptr && d->max_iters > 0 ? (d->refine_method == CTQR_REFINE_PCG ? 2 : 1) : 0;
    const bool parts = d->dtype == CTQR_F32 && refine_split_trsm<float>(d->n, smax, refine);
    L.rparts = parts ? c.take<__bf16>((int64_t)trsm_rparts_elems(d->n)) : nullptr;
    L.swork = c.take<char>(0);
    // every bucket carves the shared workspace for its own slice count: the
    // largest, or the largest that also holds the persistent kernels' exchange
    size_t sb = 0;
    for (int sl : {smax, std::min(smax, FUSED_MAX_S)})
        sb = std::max(sb, d->dtype == CTQR_F64
                              ? carve_solve<double>(nullptr, d->m, d->n, d->nb, sl, refine, false, TRSM_PARTS_X).bytes
                              : carve_solve<float>(nullptr, d->m, d->n, d->nb, sl, refine, false, TRSM_PARTS_X).bytes);
    L.bytes = c.off + sb + 256;
    return L;
}

template <typename T>
SolveRun<T> solver_run(ctqr_solver_t *sv, const SolverBucket &bk)
{
    const ctqr_solver_desc &d = sv->d;
    SolveRun<T> r = make_run<T>(d.m, d.n, (const T *)d.QR, d.lda, (const T *)d.T, (const T *)d.Rinv, d.nb,
                                sv->Bpad, sv->ldbp, bk.S, sv->refine ? &sv->sp : nullptr, d.tol,
                                sv->refine ? d.max_iters : 0, sv->swork, sv->info, false, d.refine_method,
                                TRSM_PARTS_X);
    r.narrow = bk.narrow;
    r.tp.r = sv->rparts;     // split once for the solver (solver_solve_t)
    if (!r.tp.r) r.tp.x = nullptr;
    return r;
}

void drop_graph(SolverBucket &bk)
{
    if (bk.exec) (void)hipGraphExecDestroy(bk.exec);
    bk.exec = nullptr;
}

// Captures the bucket's solve (Q^T B, the back substitution and graph_iters
// refinement iterations, no host synchronisation) on the capture stream.
template <typename T>
ctqr_status capture_bucket(ctqr_solver_t *sv, SolverBucket &bk)
{
    SolveRun<T> r = solver_run<T>(sv, bk);
    HIP_TRY(hipStreamBeginCapture(sv->cap, hipStreamCaptureModeThreadLocal));
    ctqr_status s = solve_start(r, sv->cap);
    if (!s && r.refine()) s = refine_iters(r, 0, bk.graph_iters, false, sv->cap, nullptr);
    hipGraph_t g = nullptr;
    hipError_t e = hipStreamEndCapture(sv->cap, &g);
    if (s || e != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        if (e != hipSuccess) ctqr_last_hip_error(e, "hipStreamEndCapture", __FILE__, __LINE__);
        return s ? s : CTQR_EHIP;
    }
    e = hipGraphInstantiate(&bk.exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
        bk.exec = nullptr;
        ctqr_last_hip_error(e, "hipGraphInstantiate", __FILE__, __LINE__);
        return CTQR_EHIP;
    }
    return CTQR_OK;
}

// Solves nreq requests together: their slices are packed side by side into
// the smallest bucket that holds them all (zero slices after them), solved
// once, and each request's slices copied out to its X.
template <typename T>
ctqr_status solver_solve_t(ctqr_solver_t *sv, int nreq, const double *const *B, const int64_t *ldb,
                           const int32_t *S, double *const *X, const int64_t *ldx, ctqr_info *info_out,
                           hipStream_t st)
{
    const ctqr_solver_desc &d = sv->d;
    int total = 0;
    for (int i = 0; i < nreq; ++i) total += S[i];
    SolverBucket *bp = nullptr;
    for (auto &b : sv->buckets)
        if (b.S >= total) { bp = &b; break; }
    SolverBucket &bk = *bp;
    ctqr_status s;
    // the requests into the bucket's buffer, zero slices after them (a zero
    // right-hand side gives a zero solution and leaves the others unchanged)
    for (int i = 0, off = 0; i < nreq; off += S[i], ++i)
        if ((s = copy_cm<double, double>(d.m, S[i], B[i], ldb[i], sv->Bpad + (int64_t)off * sv->ldbp, sv->ldbp,
                                         st)))
            return s;
    if (bk.S > total &&
        (s = fill_f64(sv->Bpad + (int64_t)total * sv->ldbp, (int64_t)(bk.S - total) * sv->ldbp, 0.0, st)))
        return s;
    SolveRun<T> r = solver_run<T>(sv, bk);
    if constexpr (sizeof(T) == 4) {
        // R's parts for the wide substitutions, once for the solver's life
        // (before any graph that reads them is captured or replayed)
        if (r.parts() && !sv->rparts_ready) {
            if ((s = trsm_split_r(r.n, r.QR, r.lda, sv->rparts, st))) return s;
            sv->rparts_ready = true;
        }
    }
    if (sv->refine && bk.iters < 0) {
        // calibration: an eager, host-synchronised run that counts the
        // refinement iterations the graph will hold
        if ((s = solve_start(r, st))) return s;
        int ran = 0;
        if ((s = refine_iters(r, 0, r.max_iters, true, st, &ran))) return s;
        bk.iters = ran;
        bk.graph_iters = std::min(r.max_iters, ran + GRAPH_EXTRA_ITERS);
    } else {
        if (!sv->refine) bk.graph_iters = 0;
        if (r.fused) {
            // few slices: the persistent kernels and graph_iters refinement
            // iterations, enqueued directly (a handful of launches, no graph)
            if ((s = solve_start(r, st))) return s;
            if ((s = refine_iters(r, 0, bk.graph_iters, false, st, nullptr))) return s;
            bk.direct = true;
        } else {
            if (!bk.exec && (s = capture_bucket<T>(sv, bk))) return s;
            HIP_TRY(hipGraphLaunch(bk.exec, st));
        }
        if (sv->refine && bk.graph_iters < r.max_iters) {
            // the refinement may need more iterations than the graph holds:
            // continue eagerly, and recapture with the new count next time
            bool done = false;
            if ((s = read_done(r.w.done, st, done))) return s;
            if (!done) {
                int ran = 0;
                if ((s = refine_iters(r, bk.graph_iters, r.max_iters, true, st, &ran))) return s;
                bk.iters = ran;
                bk.graph_iters = std::min(r.max_iters, ran + GRAPH_EXTRA_ITERS);
                drop_graph(bk);
            }
        }
    }
    if ((s = refine_finish(r, st))) return s;
    for (int i = 0, off = 0; i < nreq; off += S[i], ++i) {
        if (r.refine())
            s = rm_to_cm_sub(r.n, bk.S, S[i], r.w.xr + off, X[i], ldx[i], st);
        else
            s = copy_cm<double, T>(r.n, S[i], r.w.Xw + (int64_t)off * r.w.ldxw, r.w.ldxw, X[i], ldx[i], st);
        if (s) return s;
    }
    HIP_TRY(hipMemcpyAsync(info_out, sv->info, sizeof(ctqr_info), hipMemcpyDeviceToDevice, st));
    return CTQR_OK;
}

// Times Q^T B plus the back substitution of every bucket with the 32-wide
// and with the 128-wide slice tile and keeps the faster.
template <typename T>
ctqr_status solver_tune_t(ctqr_solver_t *sv, hipStream_t st, int reps)
{
    const ctqr_solver_desc &d = sv->d;
    ctqr_status s;
    if ((s = fill_f64(sv->Bpad, sv->ldbp * sv->smax, 1.0, st))) return s;
    hipEvent_t e0, e1;
    HIP_TRY(hipEventCreate(&e0));
    HIP_TRY(hipEventCreate(&e1));
    ctqr_status out = CTQR_OK;
    for (auto &bk : sv->buckets) {
        // buckets of the persistent kernels have no slice tile to choose
        if (fused_eligible<T>(d.m, d.nb, bk.S)) continue;
        const int cands[2] = {bk.S, 0};   // 32-wide, 128-wide slice tile
        const int ncand = 2;
        float best = 0.f;
        int pick = bk.narrow;
        for (int c = 0; c < ncand && !out; ++c) {
            SolveRun<T> r = make_run<T>(d.m, d.n, (const T *)d.QR, d.lda, (const T *)d.T, (const T *)d.Rinv,
                                        d.nb, sv->Bpad, sv->ldbp, bk.S, nullptr, 0.0, 0, sv->swork, sv->info,
                                        false);
            r.narrow = cands[c];
            float tot = 0.f;
            for (int rep = 0; rep <= reps && !out; ++rep) {
                hipError_t e = hipEventRecord(e0, st);
                if (e == hipSuccess && (s = solve_start(r, st))) out = s;
                if (!out && e == hipSuccess) e = hipEventRecord(e1, st);
                if (!out && e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (!out && e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) {
                    ctqr_last_hip_error(e, "solver tuning", __FILE__, __LINE__);
                    out = CTQR_EHIP;
                }
                if (rep > 0) tot += ms;   // the first run warms up
            }
            if (!out && (c == 0 || tot < best)) {
                best = tot;
                pick = cands[c];
            }
        }
        if (out) break;
        if (pick != bk.narrow) {
            bk.narrow = pick;
            bk.iters = -1;
            drop_graph(bk);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return out;
}

// Condition-number estimate: power iteration on A^T A with the FP64 sparse A
// (sigma_max), inverse iteration on R^T R through the two block substitutions
// with the factor's R (sigma_min).  Workspace layout of cond_impl.
template <typename T>
struct CondWS {
    double *x, *r, *y, *dots, *est, *dpart;   // x, r, y row-major (slice index fastest)
    T *z, *c, *yt, *w, *part;                 // column-major, leading dimension ldn
    int64_t ldn;
    size_t bytes;
};

template <typename T>
CondWS<T> carve_cond(void *work, int64_t m, int64_t n, int S)
{
    Carve c(work);
    CondWS<T> w{};
    w.ldn = round_up(n, 4);
    w.x = c.take<double>(n * S);
    w.r = c.take<double>(m * S);
    w.y = c.take<double>(n * S);
    w.dots = c.take<double>(2 * (int64_t)S);
    w.est = c.take<double>(4);
    w.dpart = c.take<double>((int64_t)slice_dot_partial_elems(S));
    w.z = c.take<T>(w.ldn * S);
    w.c = c.take<T>(w.ldn * S);
    w.yt = c.take<T>(w.ldn * S);
    w.w = c.take<T>(w.ldn * S);
    w.part = c.take<T>(SPLIT_PART_ELEMS);
    w.bytes = c.off + 256;
    return w;
}

template <typename T>
ctqr_status cond_impl(int64_t m, int64_t n, const T *QR, int64_t lda, const T *Rinv, const ctqr_sparse *A, int S,
                      int iters, void *work, double *out, hipStream_t st)
{
    CondWS<T> w = carve_cond<T>(work, m, n, S);
    NarrowScope ns(S <= DEFAULT_NARROW ? DEFAULT_NARROW : 0);
    double *q = w.dots, *nrm = w.dots + S;
    ctqr_status s;
    if ((s = fill_f64(w.est, 4, 0.0, st))) return s;
    // sigma_max(A)^2: largest Rayleigh quotient x^T A^T A x, ||x|| = 1; the
    // vectors row-major for the gathers of the sparse products
    if ((s = cond_start<double>(n, S, w.x, 0, 0x5eed0001ull, st))) return s;
    if ((s = slice_dot(n, S, w.x, w.x, w.dpart, nrm, nullptr, st))) return s;
    if ((s = rm_scale(n, S, w.x, nrm, st))) return s;
    for (int it = 0; it < iters; ++it) {
        if ((s = spmm_rowmajor(m, S, A->rowptr, A->col, A->val, 1.0, w.x, 0.0, nullptr, w.r, nullptr, st)))
            return s;
        if ((s = spmm_rowmajor(n, S, A->colptr, A->row, A->cval, 1.0, w.r, 0.0, nullptr, w.y, nullptr, st,
                               pixel_tile_side(n))))
            return s;
        if ((s = slice_dot(n, S, w.x, w.y, w.dpart, q, nullptr, st))) return s;
        if ((s = cond_max(S, q, w.est, 0, st))) return s;
        if ((s = slice_dot(n, S, w.y, w.y, w.dpart, nrm, nullptr, st))) return s;
        if ((s = rm_scale(n, S, w.y, nrm, st))) return s;
        std::swap(w.x, w.y);
    }
    // 1 / sigma_min(R)^2: largest Rayleigh quotient z^T (R^T R)^-1 z, ||z|| = 1
    if ((s = cond_start<T>(n, S, w.z, w.ldn, 0x5eed0002ull, st))) return s;
    if ((s = col_dot<T, T>(n, S, w.z, w.ldn, w.z, w.ldn, nrm, st))) return s;
    if ((s = col_scale<T, T>(n, S, w.z, w.ldn, nrm, w.z, w.ldn, st))) return s;
    for (int it = 0; it < iters; ++it) {
        // the substitutions overwrite their right-hand side: work on a copy
        if ((s = copy_cm<T, T>(n, S, w.z, w.ldn, w.c, w.ldn, st))) return s;
        s = trsm_upper_trans<T>((int)n, S, QR, lda, Rinv, w.c, w.ldn, w.yt, w.ldn, w.part, SPLIT_PART_ELEMS,
                                nullptr, st);
        if (s) return s;
        s = trsm_upper<T>((int)n, S, QR, lda, Rinv, w.yt, w.ldn, w.w, w.ldn, w.part, SPLIT_PART_ELEMS, nullptr, st);
        if (s) return s;
        if ((s = col_dot<T, T>(n, S, w.z, w.ldn, w.w, w.ldn, q, st))) return s;
        if ((s = cond_max(S, q, w.est, 1, st))) return s;
        if ((s = col_dot<T, T>(n, S, w.w, w.ldn, w.w, w.ldn, nrm, st))) return s;
        if ((s = col_scale<T, T>(n, S, w.w, w.ldn, nrm, w.z, w.ldn, st))) return s;
    }
    return cond_finish(w.est, out, st);
}

// Device address of `scratch` on the current device, looked up once per
// device with that device current.
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[NOALLOC_MAX_DEVICES] = {};

ctqr_status noalloc_scratch(void **out)
{
    int dev = -1;
    HIP_TRY(hipGetDevice(&dev));
    if (dev < 0 || dev >= NOALLOC_MAX_DEVICES) return CTQR_EUNSUPPORTED;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *p = nullptr;
        HIP_TRY(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        if (!p) return CTQR_EHIP;
        g_scratch_ptr[dev] = p;
    }
    *out = g_scratch_ptr[dev];
    return CTQR_OK;
}

bool geometry_ok(const ctqr_geometry *g)
{
    if (!g) return false;
    if (g->side < 1 || g->n_views < 1 || g->n_bins < 1) return false;
    if (g->angle_schedule != 0 && g->angle_schedule != 1) return false;
    if (g->angle_schedule == 1 && g->n_views < 4) return false;
    if (!(g->src_iso_cm > 0) || !(g->src_det_cm > g->src_iso_cm)) return false;
    if (!(g->fan_deg > 0 && g->fan_deg < 180) || !(g->fov_side_cm > 0)) return false;
    int64_t m = (int64_t)g->n_views * g->n_bins, n = (int64_t)g->side * g->side;
    return m < INT32_MAX && n < INT32_MAX;
}

// bf16 parts each block-column GEMM operand is staged as (0: FP32 MFMA)
int bf16_parts(ctqr_prec prec)
{
    return prec == CTQR_PREC_BF16_MFMA ? 1 : prec == CTQR_PREC_BF16X3_MFMA ? 2 : 0;
}

bool prec_ok(ctqr_dtype dtype, ctqr_prec prec)
{
    if (dtype == CTQR_F64) return prec == CTQR_PREC_FP64;
    if (dtype == CTQR_F32)
        return prec == CTQR_PREC_FP32_MFMA || prec == CTQR_PREC_BF16_MFMA || prec == CTQR_PREC_BF16X3_MFMA;
    return false;
}

int resolve_nb(int nb) { return nb == 0 ? DEFAULT_NB : nb; }

// The panel's row slabs of an m-row matrix fit in LDS (checked for a
// 256-CU device before any HIP call).
bool panel_fits(int m, ctqr_dtype dtype)
{
    const int rows = panel_rows_per_wg(m, 256);
    return rows <= (dtype == CTQR_F32 ? panel_max_rows_per_wg_f32() : panel_max_rows_per_wg());
}
bool nb_ok(int nb) { return nb >= 32 && nb <= 256 && nb % 32 == 0; }

}  // namespace

void ctqr_last_hip_error(hipError_t e, const char *what, const char *file, int line)
{
    char buf[512];
    snprintf(buf, sizeof buf, "%s failed: %s (%s:%d)", what, hipGetErrorString(e), file, line);
    g_last_error = buf;
}

extern "C" {

const char *ctqr_status_string(ctqr_status s)
{
    switch (s) {
    case CTQR_OK: return "CTQR_OK";
    case CTQR_EINVAL: return "CTQR_EINVAL: invalid argument";
    case CTQR_ENOMEM: return "CTQR_ENOMEM: workspace or capacity too small";
    case CTQR_EHIP: return "CTQR_EHIP: HIP runtime error";
    case CTQR_EUNSUPPORTED: return "CTQR_EUNSUPPORTED: unsupported configuration";
    case CTQR_RANK_DEFICIENT: return "CTQR_RANK_DEFICIENT: R has a negligible diagonal entry";
    case CTQR_NOT_CONVERGED: return "CTQR_NOT_CONVERGED: refinement did not converge";
    case CTQR_NONFINITE: return "CTQR_NONFINITE: NaN or Inf encountered";
    case CTQR_CAPACITY: return "CTQR_CAPACITY: sparse capacity exceeded";
    case CTQR_BARRIER_TIMEOUT: return "CTQR_BARRIER_TIMEOUT: grid barrier timed out";
    default: return "unknown ctqr status";
    }
}

const char *ctqr_version(void) { return "ctqr 0.1 gfx950"; }

const char *ctqr_last_error(void) { return g_last_error.c_str(); }

ctqr_status ctqr_geometry_sizes(const ctqr_geometry *g, int64_t *m, int64_t *n, int64_t *nnz_upper)
{
    if (!geometry_ok(g) || !m || !n || !nnz_upper) return CTQR_EINVAL;
    *m = (int64_t)g->n_views * g->n_bins;
    *n = (int64_t)g->side * g->side;
    *nnz_upper = *m * (2LL * g->side - 1);
    return CTQR_OK;
}

ctqr_status ctqr_build_workspace(const ctqr_geometry *g, size_t *bytes)
{
    if (!geometry_ok(g) || !bytes) return CTQR_EINVAL;
    *bytes = siddon_workspace(g);
    return CTQR_OK;
}

ctqr_status ctqr_build_system_matrix(const ctqr_geometry *g, ctqr_dtype dtype, void *A, int64_t lda,
                                     ctqr_sparse *sp, void *work, size_t work_bytes, ctqr_info *info,
                                     hipStream_t stream)
{
    try {
        if (!geometry_ok(g) || !info || !work) return CTQR_EINVAL;
        if (dtype != CTQR_F64 && dtype != CTQR_F32) return CTQR_EINVAL;
        const int64_t m = (int64_t)g->n_views * g->n_bins, n = (int64_t)g->side * g->side;
        if (A && (lda < m || !aligned16(A))) return CTQR_EINVAL;
        if (!A && !sp) return CTQR_EINVAL;
        if (sp) {
            if (sp->m != m || sp->n != n || sp->nnz_cap < 0 || !sp->rowptr || !sp->col || !sp->val)
                return CTQR_EINVAL;
            if ((sp->colptr != nullptr) != (sp->row != nullptr) || (sp->row != nullptr) != (sp->cval != nullptr))
                return CTQR_EINVAL;
        }
        if (work_bytes < siddon_workspace(g)) return CTQR_ENOMEM;
        ctqr_status s = info_reset(info, stream);
        if (s) return s;
        return siddon_build(g, dtype, A, lda, sp, work, work_bytes, info, stream);
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_qr_workspace(int64_t m, int64_t n, ctqr_dtype dtype, ctqr_prec prec, int32_t nb,
                              size_t *bytes)
{
    if (!bytes || m < n || n < 1 || m >= INT32_MAX) return CTQR_EINVAL;
    if (!prec_ok(dtype, prec)) return CTQR_EINVAL;
    nb = resolve_nb(nb);
    if (!nb_ok(nb)) return CTQR_EINVAL;
    *bytes = dtype == CTQR_F64 ? carve_factor<double>(nullptr, m, n, nb).bytes
                               : carve_factor<float>(nullptr, m, n, nb).bytes;
    return CTQR_OK;
}

ctqr_status ctqr_sparse_to_dense(const ctqr_sparse *sp, ctqr_dtype dtype, int64_t c0, int64_t c1, void *A,
                                 int64_t lda, hipStream_t stream)
{
    if (!sp || !sp->colptr || !sp->row || !sp->cval || !A || !aligned16(A)) return CTQR_EINVAL;
    if (dtype != CTQR_F64 && dtype != CTQR_F32) return CTQR_EINVAL;
    if (c0 < 0 || c1 < c0 || c1 > sp->n || lda < sp->m || sp->n >= INT32_MAX) return CTQR_EINVAL;
    return sparse_to_dense_cols(sp, dtype, (int)c0, (int)c1, A, lda, stream);
}

ctqr_status ctqr_qr_factor_ooc_workspace(int64_t m, int64_t n, ctqr_dtype dtype, ctqr_prec prec, int32_t nb,
                                         int64_t lda, int64_t tile_cols, size_t *bytes)
{
    if (!bytes || m < n || n < 1 || m >= INT32_MAX || lda < m || tile_cols < 1) return CTQR_EINVAL;
    if (!prec_ok(dtype, prec)) return CTQR_EINVAL;
    nb = resolve_nb(nb);
    if (!nb_ok(nb)) return CTQR_EINVAL;
    *bytes = dtype == CTQR_F64 ? carve_ooc<double>(nullptr, m, n, nb, lda, tile_cols).bytes
                               : carve_ooc<float>(nullptr, m, n, nb, lda, tile_cols).bytes;
    return CTQR_OK;
}

ctqr_status ctqr_qr_factor_ooc(int64_t m, int64_t n, ctqr_dtype dtype, void *A_dev, void *A_host, int64_t lda,
                               int64_t n_dev, int64_t tile_cols, ctqr_prec prec, int32_t nb, void *T, double *tau,
                               void *Rinv, void *work, size_t work_bytes, ctqr_info *info, hipStream_t stream)
{
    try {
        if (m < n || n < 1 || m >= INT32_MAX || !T || !tau || !work || !info) return CTQR_EINVAL;
        if (lda < m || lda % 4 != 0 || !aligned16(T) || !aligned16(work)) return CTQR_EINVAL;
        if (Rinv && !aligned16(Rinv)) return CTQR_EINVAL;
        if (!prec_ok(dtype, prec))
            return CTQR_EINVAL;
        nb = resolve_nb(nb);
        if (!nb_ok(nb)) return CTQR_EINVAL;
        // block boundaries: resident part and tiles are whole 2048-column
        // diagonal blocks of the substitution and whole nb-column blocks
        if (n_dev < 0 || n_dev > n || tile_cols < 1) return CTQR_EINVAL;
        if (n_dev % TRSM_BIG != 0 || n_dev % nb != 0 || tile_cols % TRSM_BIG != 0 || tile_cols % nb != 0)
            return CTQR_EINVAL;
        if (n_dev > 0 && (!A_dev || !aligned16(A_dev))) return CTQR_EINVAL;
        if (n_dev < n && (!A_host || !aligned16(A_host))) return CTQR_EINVAL;
        size_t need = 0;
        ctqr_qr_factor_ooc_workspace(m, n, dtype, prec, nb, lda, tile_cols, &need);
        if (work_bytes < need) return CTQR_ENOMEM;
        if (!panel_fits((int)m, dtype)) return CTQR_EUNSUPPORTED;
        if (n_dev < n) {
            // the host part must be pinned (page-locked) host memory
            hipPointerAttribute_t at{};
            if (hipPointerGetAttributes(&at, A_host) != hipSuccess || at.type != hipMemoryTypeHost) {
                (void)hipGetLastError();
                return CTQR_EINVAL;
            }
        }
        ctqr_status s = ensure_setup();
        if (s) return s;
        if (dtype == CTQR_F64)
            return factor_ooc_impl<double>(m, n, (double *)A_dev, (double *)A_host, lda, n_dev, tile_cols, nb,
                                           (double *)T, tau, (double *)Rinv, work, info, stream, 0);
        return factor_ooc_impl<float>(m, n, (float *)A_dev, (float *)A_host, lda, n_dev, tile_cols, nb, (float *)T,
                                      tau, (float *)Rinv, work, info, stream, bf16_parts(prec));
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_qr_rinv_bytes(int64_t n, ctqr_dtype dtype, size_t *bytes)
{
    if (!bytes || n < 1 || n >= INT32_MAX || (dtype != CTQR_F64 && dtype != CTQR_F32)) return CTQR_EINVAL;
    *bytes = 2 * trinv_elems((int)n) * (dtype == CTQR_F64 ? sizeof(double) : sizeof(float));
    return CTQR_OK;
}

ctqr_status ctqr_qr_factor(int64_t m, int64_t n, ctqr_dtype dtype, void *A, int64_t lda, ctqr_prec prec,
                           int32_t nb, void *T, double *tau, void *Rinv, void *work, size_t work_bytes,
                           ctqr_info *info, hipStream_t stream)
{
    try {
        if (m < n || n < 1 || m >= INT32_MAX || !A || !T || !tau || !work || !info) return CTQR_EINVAL;
        if (lda < m || lda % 4 != 0 || !aligned16(A) || !aligned16(T)) return CTQR_EINVAL;
        if (Rinv && !aligned16(Rinv)) return CTQR_EINVAL;
        if (!prec_ok(dtype, prec))
            return CTQR_EINVAL;
        nb = resolve_nb(nb);
        if (!nb_ok(nb)) return CTQR_EINVAL;
        size_t need = 0;
        ctqr_qr_workspace(m, n, dtype, prec, nb, &need);
        if (work_bytes < need || !aligned16(work)) return work_bytes < need ? CTQR_ENOMEM : CTQR_EINVAL;
        if (!panel_fits((int)m, dtype)) return CTQR_EUNSUPPORTED;
        ctqr_status s = ensure_setup();
        if (s) return s;
        if (dtype == CTQR_F64)
            return factor_impl<double>(m, n, (double *)A, lda, nb, (double *)T, tau, (double *)Rinv, work, info,
                                       stream, 0);
        return factor_impl<float>(m, n, (float *)A, lda, nb, (float *)T, tau, (float *)Rinv, work, info, stream,
                                  bf16_parts(prec));
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_qr_tune_nb(int64_t m, int64_t n, ctqr_dtype dtype, void *A, int64_t lda, ctqr_prec prec, void *T,
                           double *tau, void *work, size_t work_bytes, ctqr_info *info, int32_t *nb_best,
                           float *ms_per_col, hipStream_t stream)
{
    try {
        if (m < n || n < 1 || m >= INT32_MAX || !A || !T || !tau || !work || !info || !nb_best) return CTQR_EINVAL;
        if (lda < m || lda % 4 != 0 || !aligned16(A) || !aligned16(T)) return CTQR_EINVAL;
        if (!prec_ok(dtype, prec)) return CTQR_EINVAL;
        size_t need = 0;
        ctqr_qr_workspace(m, n, dtype, prec, TUNE_NB[2], &need);
        if (work_bytes < need || !aligned16(work)) return work_bytes < need ? CTQR_ENOMEM : CTQR_EINVAL;
        if (!panel_fits((int)m, dtype)) return CTQR_EUNSUPPORTED;
        ctqr_status s = ensure_setup();
        if (s) return s;
        if (dtype == CTQR_F64)
            return tune_nb_impl<double>(m, n, (double *)A, lda, (double *)T, tau, work, info, stream, 0, nb_best,
                                        ms_per_col);
        return tune_nb_impl<float>(m, n, (float *)A, lda, (float *)T, tau, work, info, stream, bf16_parts(prec),
                                   nb_best, ms_per_col);
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_solve_workspace(int64_t m, int64_t n, ctqr_dtype dtype, int32_t nb, int32_t nslices,
                                 int32_t refine, size_t *bytes)
{
    if (!bytes || m < n || n < 1 || m >= INT32_MAX || nslices < 1) return CTQR_EINVAL;
    if (dtype != CTQR_F64 && dtype != CTQR_F32) return CTQR_EINVAL;
    nb = resolve_nb(nb);
    if (!nb_ok(nb)) return CTQR_EINVAL;
    if (refine < 0 || refine > 2) return CTQR_EINVAL;
    *bytes = dtype == CTQR_F64 ? carve_solve<double>(nullptr, m, n, nb, nslices, refine, true, TRSM_PARTS_ALL).bytes
                               : carve_solve<float>(nullptr, m, n, nb, nslices, refine, true, TRSM_PARTS_ALL).bytes;
    return CTQR_OK;
}

ctqr_status ctqr_qr_solve_slices(int64_t m, int64_t n, ctqr_dtype dtype, const void *QR, int64_t lda,
                                 const void *T, const double *tau, const void *Rinv, int32_t nb, const double *B,
                                 int64_t ldb, int32_t nslices, double *X, int64_t ldx,
                                 const ctqr_sparse *A64, double tol, int32_t max_iters, int32_t refine_method,
                                 void *work, size_t work_bytes, ctqr_info *info, hipStream_t stream)
{
    try {
        if (m < n || n < 1 || m >= INT32_MAX || nslices < 1) return CTQR_EINVAL;
        if (!QR || !T || !tau || !B || !X || !work || !info) return CTQR_EINVAL;
        if (refine_method != CTQR_REFINE_CSNE && refine_method != CTQR_REFINE_PCG) return CTQR_EINVAL;
        if (dtype != CTQR_F64 && dtype != CTQR_F32) return CTQR_EINVAL;
        if (lda < m || lda % 4 != 0 || ldb < m || ldx < n) return CTQR_EINVAL;
        if (!aligned16(QR) || !aligned16(T) || !aligned16(work)) return CTQR_EINVAL;
        nb = resolve_nb(nb);
        if (!nb_ok(nb)) return CTQR_EINVAL;
        if (A64 && (A64->m != m || A64->n != n || !A64->rowptr || !A64->col || !A64->val ||
                    !A64->colptr || !A64->row || !A64->cval))
            return CTQR_EINVAL;
        if (A64 && (max_iters < 0 || !(tol >= 0.0))) return CTQR_EINVAL;
        size_t need = 0;
        const int refine = A64 != nullptr && max_iters > 0 ? (refine_method == CTQR_REFINE_PCG ? 2 : 1) : 0;
        ctqr_solve_workspace(m, n, dtype, nb, nslices, refine, &need);
        if (work_bytes < need) return CTQR_ENOMEM;
        if (Rinv && !aligned16(Rinv)) return CTQR_EINVAL;
        if (dtype == CTQR_F64)
            return solve_impl<double>(m, n, (const double *)QR, lda, (const double *)T, tau, (const double *)Rinv,
                                      nb, B, ldb, nslices, X, ldx, A64, tol, max_iters, refine_method, work, info,
                                      stream);
        return solve_impl<float>(m, n, (const float *)QR, lda, (const float *)T, tau, (const float *)Rinv, nb, B,
                                 ldb, nslices, X, ldx, A64, tol, max_iters, refine_method, work, info, stream);
    } catch (...) {
        return CTQR_EHIP;
    }
}

namespace {
ctqr_status ctqr_qr_solve_slices_noalloc(int64_t m, int64_t n, ctqr_dtype dtype, const void *QR, int64_t lda,
                                         const void *T, const double *tau, const void *Rinv, int32_t nb,
                                         const double *B, int64_t ldb, int32_t nslices, double *X, int64_t ldx,
                                         const ctqr_sparse *A64, double tol, int32_t max_iters,
                                         int32_t refine_method, ctqr_info *info, hipStream_t stream)
{
    try {
        if (m < n || n < 1 || m >= INT32_MAX || nslices < 1) return CTQR_EINVAL;
        if (!QR || !T || !tau || !B || !X || !info) return CTQR_EINVAL;
        if (refine_method != CTQR_REFINE_CSNE && refine_method != CTQR_REFINE_PCG) return CTQR_EINVAL;
        if (dtype != CTQR_F64 && dtype != CTQR_F32) return CTQR_EINVAL;
        if (lda < m || lda % 4 != 0 || ldb < m || ldx < n) return CTQR_EINVAL;
        if (!aligned16(QR) || !aligned16(T)) return CTQR_EINVAL;
        nb = resolve_nb(nb);
        if (!nb_ok(nb)) return CTQR_EINVAL;
        if (A64 && (A64->m != m || A64->n != n || !A64->rowptr || !A64->col || !A64->val ||
                    !A64->colptr || !A64->row || !A64->cval))
            return CTQR_EINVAL;
        if (A64 && (max_iters < 0 || !(tol >= 0.0))) return CTQR_EINVAL;
        if (Rinv && !aligned16(Rinv)) return CTQR_EINVAL;
        // the same workspace layout as ctqr_qr_solve_slices, in the scratch
        size_t need = 0;
        const int refine = A64 != nullptr && max_iters > 0 ? (refine_method == CTQR_REFINE_PCG ? 2 : 1) : 0;
        ctqr_status s = ctqr_solve_workspace(m, n, dtype, nb, nslices, refine, &need);
        if (s) return s;
        if (need > CTQR_NOALLOC_SCRATCH_BYTES) {
            g_last_error = "ctqr_qr_solve_slices_noalloc: the solve needs " + std::to_string(need) +
                           " bytes of scratch, more than CTQR_NOALLOC_SCRATCH_BYTES (" +
                           std::to_string((size_t)CTQR_NOALLOC_SCRATCH_BYTES) + ")";
            return CTQR_ENOMEM;
        }
        void *work = nullptr;
        if ((s = noalloc_scratch(&work))) return s;
        struct NoAlloc {
            NoAlloc() { t_no_alloc = true; }
            ~NoAlloc() { t_no_alloc = false; }
        } no_alloc;
        if (dtype == CTQR_F64)
            return solve_impl<double>(m, n, (const double *)QR, lda, (const double *)T, tau, (const double *)Rinv,
                                      nb, B, ldb, nslices, X, ldx, A64, tol, max_iters, refine_method, work, info,
                                      stream, true);
        return solve_impl<float>(m, n, (const float *)QR, lda, (const float *)T, tau, (const float *)Rinv, nb, B,
                                 ldb, nslices, X, ldx, A64, tol, max_iters, refine_method, work, info, stream, true);
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status solver_desc_check(const ctqr_solver_desc *d)
{
    if (!d) return CTQR_EINVAL;
    if (d->m < d->n || d->n < 1 || d->m >= INT32_MAX) return CTQR_EINVAL;
    if (d->dtype != CTQR_F64 && d->dtype != CTQR_F32) return CTQR_EINVAL;
    if (!nb_ok(resolve_nb(d->nb))) return CTQR_EINVAL;
    if (!d->QR || !d->T || !d->tau || !d->Rinv) return CTQR_EINVAL;
    if (!aligned16(d->QR) || !aligned16(d->T) || !aligned16(d->Rinv)) return CTQR_EINVAL;
    if (d->lda < d->m || d->lda % 4 != 0) return CTQR_EINVAL;
    if (d->max_slices < 1 || d->max_slices > SOLVER_MAX_SLICES) return CTQR_EINVAL;
    const ctqr_sparse *A = d->A64;
    if (A && (A->m != d->m || A->n != d->n || !A->rowptr || !A->col || !A->val || !A->colptr || !A->row ||
              !A->cval))
        return CTQR_EINVAL;
    if (A && (d->max_iters < 0 || !(d->tol >= 0.0))) return CTQR_EINVAL;
    if (d->refine_method != CTQR_REFINE_CSNE && d->refine_method != CTQR_REFINE_PCG) return CTQR_EINVAL;
    return CTQR_OK;
}
}  // namespace

ctqr_status ctqr_solver_workspace(const ctqr_solver_desc *desc, size_t *bytes)
{
    ctqr_status s = solver_desc_check(desc);
    if (s || !bytes) return s ? s : CTQR_EINVAL;
    ctqr_solver_desc d = *desc;
    d.nb = resolve_nb(d.nb);
    *bytes = solver_layout(&d, nullptr, bucket_cap(d.max_slices), round_up(d.m, 64)).bytes;
    return CTQR_OK;
}

ctqr_status ctqr_solver_create(const ctqr_solver_desc *desc, void *work, size_t work_bytes, ctqr_solver *out)
{
    try {
        ctqr_status s = solver_desc_check(desc);
        if (s) return s;
        if (!out || !work || !aligned16(work)) return CTQR_EINVAL;
        *out = nullptr;
        size_t need = 0;
        ctqr_solver_workspace(desc, &need);
        if (work_bytes < need) return CTQR_ENOMEM;
        auto *sv = new ctqr_solver_t;
        sv->d = *desc;
        sv->d.nb = resolve_nb(desc->nb);
        sv->refine = desc->A64 != nullptr && desc->max_iters > 0;
        if (desc->A64) sv->sp = *desc->A64;
        sv->d.A64 = desc->A64 ? &sv->sp : nullptr;
        sv->smax = bucket_cap(desc->max_slices);
        sv->ldbp = round_up(desc->m, 64);
        SolverLayout L = solver_layout(&sv->d, work, sv->smax, sv->ldbp);
        sv->info = L.info;
        sv->Bpad = L.Bpad;
        sv->rparts = L.rparts;
        sv->swork = L.swork;
        for (int b : bucket_sizes(sv->smax)) {
            SolverBucket bk;
            bk.S = b;
            bk.narrow = b <= DEFAULT_NARROW ? DEFAULT_NARROW : 0;
            sv->buckets.push_back(bk);
        }
        hipError_t e = hipStreamCreateWithFlags(&sv->cap, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sv->last, hipEventDisableTiming);
        if (e != hipSuccess) {
            ctqr_last_hip_error(e, "solver stream and event", __FILE__, __LINE__);
            if (sv->cap) (void)hipStreamDestroy(sv->cap);
            delete sv;
            return CTQR_EHIP;
        }
        *out = sv;
        return CTQR_OK;
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_solver_tune(ctqr_solver sv, int32_t reps, hipStream_t stream)
{
    try {
        if (!sv || reps < 1 || reps > 100) return CTQR_EINVAL;
        std::lock_guard<std::mutex> lk(sv->mu);
        SolverOrder ord{sv, stream};
        ctqr_status s = ord.begin();
        if (s) return s;
        s = sv->d.dtype == CTQR_F64 ? solver_tune_t<double>(sv, stream, reps) : solver_tune_t<float>(sv, stream, reps);
        ctqr_status e = ord.end();
        return s ? s : e;
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_solver_solve(ctqr_solver sv, const double *B, int64_t ldb, int32_t nslices, double *X,
                              int64_t ldx, ctqr_info *info, hipStream_t stream)
{
    return ctqr_solver_solve_batch(sv, 1, &B, &ldb, &nslices, &X, &ldx, info, stream);
}

ctqr_status ctqr_solver_solve_batch(ctqr_solver sv, int32_t nreq, const double *const *B, const int64_t *ldb,
                                    const int32_t *nslices, double *const *X, const int64_t *ldx, ctqr_info *info,
                                    hipStream_t stream)
{
    try {
        if (!sv || nreq < 1 || !B || !ldb || !nslices || !X || !ldx || !info) return CTQR_EINVAL;
        int64_t total = 0;
        for (int i = 0; i < nreq; ++i) {
            if (!B[i] || !X[i] || nslices[i] < 1 || ldb[i] < sv->d.m || ldx[i] < sv->d.n) return CTQR_EINVAL;
            total += nslices[i];
        }
        if (total > sv->smax) return CTQR_EINVAL;
        std::lock_guard<std::mutex> lk(sv->mu);
        SolverOrder ord{sv, stream};
        ctqr_status s = ord.begin();
        if (s) return s;
        s = sv->d.dtype == CTQR_F64 ? solver_solve_t<double>(sv, nreq, B, ldb, nslices, X, ldx, info, stream)
                                    : solver_solve_t<float>(sv, nreq, B, ldb, nslices, X, ldx, info, stream);
        ctqr_status e = ord.end();
        return s ? s : e;
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_solver_query(ctqr_solver sv, int32_t nslices, int32_t *bucket, int32_t *slice_tile,
                              int32_t *graph_iters)
{
    if (!sv || !bucket || !slice_tile || !graph_iters || nslices < 1 || nslices > sv->smax) return CTQR_EINVAL;
    std::lock_guard<std::mutex> lk(sv->mu);
    for (auto &b : sv->buckets)
        if (b.S >= nslices) {
            *bucket = b.S;
            *slice_tile = b.narrow >= b.S ? 32 : 128;
            *graph_iters = b.exec || b.direct ? b.graph_iters : -1;
            return CTQR_OK;
        }
    return CTQR_EINVAL;
}

ctqr_status ctqr_solver_destroy(ctqr_solver sv)
{
    if (!sv) return CTQR_OK;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        for (auto &b : sv->buckets) drop_graph(b);
        if (sv->cap) (void)hipStreamDestroy(sv->cap);
        if (sv->last) (void)hipEventDestroy(sv->last);
    }
    delete sv;
    return CTQR_OK;
}

ctqr_status ctqr_solve_ooc_workspace(int64_t m, int64_t n, ctqr_dtype dtype, int32_t nb, int32_t nslices,
                                     int32_t refine, int64_t lda, int64_t tile_cols, size_t *bytes)
{
    if (!bytes || m < n || n < 1 || m >= INT32_MAX || nslices < 1 || lda < m || tile_cols < 1) return CTQR_EINVAL;
    if (dtype != CTQR_F64 && dtype != CTQR_F32) return CTQR_EINVAL;
    nb = resolve_nb(nb);
    if (!nb_ok(nb)) return CTQR_EINVAL;
    const size_t esz = dtype == CTQR_F64 ? sizeof(double) : sizeof(float);
    if (refine < 0 || refine > 2) return CTQR_EINVAL;
    const size_t sb = dtype == CTQR_F64 ? carve_solve<double>(nullptr, m, n, nb, nslices, refine, false).bytes
                                        : carve_solve<float>(nullptr, m, n, nb, nslices, refine, false).bytes;
    *bytes = sb + 256 + (size_t)lda * (size_t)tile_cols * esz + 256;
    return CTQR_OK;
}

ctqr_status ctqr_qr_solve_ooc(int64_t m, int64_t n, ctqr_dtype dtype, const void *QR_dev, const void *QR_host,
                              int64_t lda, int64_t n_dev, int64_t tile_cols, const void *T, const double *tau,
                              const void *Rinv, int32_t nb, const double *B, int64_t ldb, int32_t nslices, double *X,
                              int64_t ldx, const ctqr_sparse *A64, double tol, int32_t max_iters,
                              int32_t refine_method, void *work, size_t work_bytes, ctqr_info *info,
                              hipStream_t stream)
{
    try {
        if (m < n || n < 1 || m >= INT32_MAX || nslices < 1) return CTQR_EINVAL;
        if (!T || !tau || !Rinv || !B || !X || !work || !info) return CTQR_EINVAL;
        if (refine_method != CTQR_REFINE_CSNE && refine_method != CTQR_REFINE_PCG) return CTQR_EINVAL;
        if (dtype != CTQR_F64 && dtype != CTQR_F32) return CTQR_EINVAL;
        if (lda < m || lda % 4 != 0 || ldb < m || ldx < n) return CTQR_EINVAL;
        if (!aligned16(T) || !aligned16(Rinv) || !aligned16(work)) return CTQR_EINVAL;
        nb = resolve_nb(nb);
        if (!nb_ok(nb)) return CTQR_EINVAL;
        if (n_dev < 0 || n_dev > n || tile_cols < 1) return CTQR_EINVAL;
        if (n_dev % TRSM_BIG != 0 || n_dev % nb != 0 || tile_cols % TRSM_BIG != 0 || tile_cols % nb != 0)
            return CTQR_EINVAL;
        if (n_dev > 0 && (!QR_dev || !aligned16(QR_dev))) return CTQR_EINVAL;
        if (n_dev < n && (!QR_host || !aligned16(QR_host))) return CTQR_EINVAL;
        if (A64 && (A64->m != m || A64->n != n || !A64->rowptr || !A64->col || !A64->val || !A64->colptr ||
                    !A64->row || !A64->cval))
            return CTQR_EINVAL;
        if (A64 && (max_iters < 0 || !(tol >= 0.0))) return CTQR_EINVAL;
        size_t need = 0;
        const int refine = A64 != nullptr && max_iters > 0 ? (refine_method == CTQR_REFINE_PCG ? 2 : 1) : 0;
        ctqr_solve_ooc_workspace(m, n, dtype, nb, nslices, refine, lda, tile_cols, &need);
        if (work_bytes < need) return CTQR_ENOMEM;
        if (n_dev < n) {
            hipPointerAttribute_t at{};
            if (hipPointerGetAttributes(&at, QR_host) != hipSuccess || at.type != hipMemoryTypeHost) {
                (void)hipGetLastError();
                return CTQR_EINVAL;
            }
        }
        if (dtype == CTQR_F64)
            return solve_ooc_impl<double>(m, n, (const double *)QR_dev, (const double *)QR_host, lda, (int)n_dev,
                                          (int)tile_cols, (const double *)T, (const double *)Rinv, nb, B, ldb, nslices,
                                          X, ldx, A64, tol, max_iters, refine_method, work, info, stream);
        return solve_ooc_impl<float>(m, n, (const float *)QR_dev, (const float *)QR_host, lda, (int)n_dev,
                                     (int)tile_cols, (const float *)T, (const float *)Rinv, nb, B, ldb, nslices, X,
                                     ldx, A64, tol, max_iters, refine_method, work, info, stream);
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_cond_workspace(int64_t m, int64_t n, ctqr_dtype dtype, int32_t nvec, size_t *bytes)
{
    if (!bytes || m < n || n < 1 || nvec < 1 || nvec > 64) return CTQR_EINVAL;
    if (dtype == CTQR_F64)
        *bytes = carve_cond<double>(nullptr, m, n, nvec).bytes;
    else if (dtype == CTQR_F32)
        *bytes = carve_cond<float>(nullptr, m, n, nvec).bytes;
    else
        return CTQR_EINVAL;
    return CTQR_OK;
}

ctqr_status ctqr_cond_estimate(int64_t m, int64_t n, ctqr_dtype dtype, const void *QR, int64_t lda, const void *Rinv,
                               const ctqr_sparse *A64, int32_t nvec, int32_t iters, void *work, size_t work_bytes,
                               double *out, hipStream_t stream)
{
    try {
        size_t need = 0;
        ctqr_status s = ctqr_cond_workspace(m, n, dtype, nvec, &need);
        if (s) return s;
        if (!QR || !Rinv || !A64 || !work || !out || iters < 1 || m >= INT32_MAX) return CTQR_EINVAL;
        if (lda < m || lda % 4 || !aligned16(QR)) return CTQR_EINVAL;
        if (A64->m != m || A64->n != n || !A64->rowptr || !A64->col || !A64->val || !A64->colptr || !A64->row ||
            !A64->cval)
            return CTQR_EINVAL;
        if (!aligned16(work) || !aligned16(Rinv)) return CTQR_EINVAL;
        if (work_bytes < need) return CTQR_ENOMEM;
        if (dtype == CTQR_F64)
            return cond_impl<double>(m, n, (const double *)QR, lda, (const double *)Rinv, A64, nvec, iters, work,
                                     out, stream);
        return cond_impl<float>(m, n, (const float *)QR, lda, (const float *)Rinv, A64, nvec, iters, work, out,
                                stream);
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_tile_tasks(int32_t mt, int32_t nt, int32_t solve, ctqr_tile_task *tasks, int64_t cap,
                            int64_t *count)
{
    try {
        if (mt < 1 || nt < 1 || mt < nt || !count || (solve != 0 && solve != 1) || (tasks && cap < 0))
            return CTQR_EINVAL;
        const std::vector<int4> v = solve ? tile_solve_tasks(mt, nt) : tile_qr_tasks(mt, nt);
        *count = (int64_t)v.size();
        if (tasks)
            for (int64_t q = 0; q < std::min<int64_t>(cap, (int64_t)v.size()); ++q)
                tasks[q] = ctqr_tile_task{v[q].x, v[q].y, v[q].z, v[q].w};
        return CTQR_OK;
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_tile_qr_sizes(int64_t m, int64_t n, int32_t b, int64_t *s_elems, size_t *work_bytes)
{
    if (!s_elems || !work_bytes || m < n || n < 1 || b < 1 || b > 64 || m >= INT32_MAX) return CTQR_EINVAL;
    const int64_t mt = ceil_div(m, b), nt = ceil_div(n, b);
    *s_elems = mt * nt * (int64_t)b * b;
    // apply tasks of the factorization: sum over j of sum_{k<j} (mt - k); plus
    // the factor tasks; the solve has fewer
    int64_t cnt = 0;
    for (int64_t j = 0; j < nt; ++j) cnt += j * mt - j * (j - 1) / 2 + (mt - j);
    const int64_t scnt = nt * mt - nt * (nt - 1) / 2 + nt * (nt + 1) / 2;
    *work_bytes = (size_t)std::max(cnt, scnt) * 16 + 256;
    return CTQR_OK;
}

ctqr_status ctqr_tile_qr_factor(int64_t m, int64_t n, double *A, int64_t lda, int32_t b, double *S, void *work,
                                size_t work_bytes, hipStream_t stream)
{
    try {
        int64_t se = 0;
        size_t wb = 0;
        ctqr_status s = ctqr_tile_qr_sizes(m, n, b, &se, &wb);
        if (s) return s;
        if (!A || !S || !work || lda < m) return CTQR_EINVAL;
        if (work_bytes < wb) return CTQR_ENOMEM;
        return tile_qr_run((int)m, (int)n, b, A, lda, S, (int4 *)work, stream);
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_tile_qr_solve(int64_t m, int64_t n, const double *QR, int64_t lda, int32_t b, const double *S,
                               double *B, int64_t ldb, int32_t nslices, void *work, size_t work_bytes,
                               hipStream_t stream)
{
    try {
        int64_t se = 0;
        size_t wb = 0;
        ctqr_status s = ctqr_tile_qr_sizes(m, n, b, &se, &wb);
        if (s) return s;
        if (!QR || !S || !B || !work || lda < m || ldb < m || nslices < 1) return CTQR_EINVAL;
        if (work_bytes < wb) return CTQR_ENOMEM;
        return tile_solve_run((int)m, (int)n, b, QR, lda, S, B, ldb, nslices, (int4 *)work, stream);
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_project_joseph(const ctqr_geometry *g, int32_t nslices, const double *X, int64_t ldx, double *B,
                                int64_t ldb, hipStream_t stream)
{
    try {
        if (!geometry_ok(g) || !X || !B || nslices < 1) return CTQR_EINVAL;
        const int64_t m = (int64_t)g->n_views * g->n_bins, n = (int64_t)g->side * g->side;
        if (ldx < n || ldb < m || m >= INT32_MAX) return CTQR_EINVAL;
        return joseph_project(g, nslices, X, ldx, B, ldb, stream);
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_image_quality(int32_t side, int32_t nslices, const double *Xref, int64_t ldr, const double *X,
                               int64_t ldx, double data_range, double *out, hipStream_t stream)
{
    try {
        if (side < 1 || nslices < 1 || !Xref || !X || !out || !(data_range >= 0.0)) return CTQR_EINVAL;
        const int64_t n = (int64_t)side * side;
        if (ldr < n || ldx < n) return CTQR_EINVAL;
        return image_quality(side, nslices, Xref, ldr, X, ldx, data_range, out, stream);
    } catch (...) {
        return CTQR_EHIP;
    }
}

// ---- View-count search -------------------------------------------------------
namespace {
struct ViewSearchWS {
    ctqr_info *info;
    double *out, *A, *T, *tau, *Rinv, *val, *cval;
    int64_t *rowptr, *colptr;
    int32_t *col, *row;
    void *qrwork, *bwork, *cwork;
    size_t qrbytes, bbytes, cbytes, bytes;
    int64_t lda, cap;
};

constexpr int VIEW_NB = 256;
constexpr int VIEW_NVEC = 8;

ViewSearchWS carve_view_search(void *work, const ctqr_geometry *g, int v_max)
{
    ctqr_geometry gm = *g;
    gm.n_views = v_max;
    const int64_t m = (int64_t)v_max * g->n_bins, n = (int64_t)g->side * g->side;
    Carve c(work);
    ViewSearchWS w{};
    w.lda = round_up(m, 64);
    w.cap = m * (2LL * g->side - 1);
    w.info = c.take<ctqr_info>(1);
    w.out = c.take<double>(4);
    w.A = c.take<double>(w.lda * n);
    w.T = c.take<double>((int64_t)VIEW_NB * n);
    w.tau = c.take<double>(n);
    w.Rinv = c.take<double>(2 * (int64_t)trinv_elems((int)n));
    w.rowptr = c.take<int64_t>(m + 1);
    w.col = c.take<int32_t>(w.cap);
    w.val = c.take<double>(w.cap);
    w.colptr = c.take<int64_t>(n + 1);
    w.row = c.take<int32_t>(w.cap);
    w.cval = c.take<double>(w.cap);
    w.qrbytes = 0;
    if (m >= n) (void)ctqr_qr_workspace(m, n, CTQR_F64, CTQR_PREC_FP64, VIEW_NB, &w.qrbytes);
    w.qrwork = c.take<char>((int64_t)w.qrbytes);
    w.bbytes = siddon_workspace(&gm);
    w.bwork = c.take<char>((int64_t)w.bbytes);
    w.cbytes = 0;
    if (m >= n) (void)ctqr_cond_workspace(m, n, CTQR_F64, VIEW_NVEC, &w.cbytes);
    w.cwork = c.take<char>((int64_t)w.cbytes);
    w.bytes = c.off + 256;
    return w;
}
}  // namespace

ctqr_status ctqr_view_search_workspace(const ctqr_geometry *g, int32_t v_max, size_t *bytes)
{
    if (!bytes || !g || v_max < 1) return CTQR_EINVAL;
    ctqr_geometry gm = *g;
    gm.n_views = v_max;
    if (!geometry_ok(&gm)) return CTQR_EINVAL;
    *bytes = carve_view_search(nullptr, g, v_max).bytes;
    return CTQR_OK;
}

ctqr_status ctqr_view_search(const ctqr_geometry *g, int32_t v_min, int32_t v_max, int32_t v_step, double kappa_max,
                             int32_t iters, void *work, size_t work_bytes, ctqr_view_trial *trials,
                             int32_t max_trials, int32_t *n_trials, int32_t *v_best, hipStream_t stream)
{
    try {
        if (!g || !work || !trials || !n_trials || !v_best || v_min < 1 || v_max < v_min || v_step < 1 ||
            max_trials < 1 || iters < 1 || !(kappa_max > 1.0))
            return CTQR_EINVAL;
        size_t need = 0;
        ctqr_status s = ctqr_view_search_workspace(g, v_max, &need);
        if (s) return s;
        if (work_bytes < need || !aligned16(work)) return work_bytes < need ? CTQR_ENOMEM : CTQR_EINVAL;
        ViewSearchWS w = carve_view_search(work, g, v_max);
        const int64_t n = (int64_t)g->side * g->side;
        *n_trials = 0;
        *v_best = 0;
        for (int v = v_min; v <= v_max && *n_trials < max_trials; v += v_step) {
            ctqr_geometry gv = *g;
            gv.n_views = v;
            const int64_t m = (int64_t)v * g->n_bins;
            ctqr_view_trial &t = trials[(*n_trials)++];
            t.views = v;
            t.status = CTQR_RANK_DEFICIENT;
            t.kappa = INFINITY;
            t.rdiag_min = t.rdiag_max = 0.0;
            if (m < n) continue;   // fewer rays than pixels: never full column rank
            if (!panel_fits((int)m, CTQR_F64)) return CTQR_EUNSUPPORTED;
            ctqr_sparse sp{m, n, w.cap, w.rowptr, w.col, w.val, w.colptr, w.row, w.cval};
            if ((s = ctqr_build_system_matrix(&gv, CTQR_F64, w.A, w.lda, &sp, w.bwork, w.bbytes, w.info, stream)))
                return s;
            ctqr_info bi{};
            HIP_TRY(hipMemcpyAsync(&bi, w.info, sizeof(bi), hipMemcpyDeviceToHost, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            if (bi.status) return CTQR_ENOMEM;   // sparse capacity: cannot happen with the upper bound
            size_t qb = 0;
            if ((s = ctqr_qr_workspace(m, n, CTQR_F64, CTQR_PREC_FP64, VIEW_NB, &qb))) return s;
            if ((s = ctqr_qr_factor(m, n, CTQR_F64, w.A, w.lda, CTQR_PREC_FP64, VIEW_NB, w.T, w.tau, w.Rinv,
                                    w.qrwork, w.qrbytes, w.info, stream)))
                return s;
            ctqr_info fi{};
            HIP_TRY(hipMemcpyAsync(&fi, w.info, sizeof(fi), hipMemcpyDeviceToHost, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            t.rdiag_min = fi.rdiag_min;
            t.rdiag_max = fi.rdiag_max;
            if (fi.status == CTQR_NONFINITE || fi.status == CTQR_BARRIER_TIMEOUT) return CTQR_EHIP;
            if ((s = ctqr_cond_estimate(m, n, CTQR_F64, w.A, w.lda, w.Rinv, &sp, VIEW_NVEC, iters, w.cwork, w.cbytes,
                                        w.out, stream)))
                return s;
            double est[3] = {0, 0, 0};
            HIP_TRY(hipMemcpyAsync(est, w.out, sizeof(est), hipMemcpyDeviceToHost, stream));
            HIP_TRY(hipStreamSynchronize(stream));
            t.kappa = est[2];
            if (fi.status == 0 && est[2] <= kappa_max) {
                t.status = CTQR_OK;
                *v_best = v;
                break;
            }
        }
        return CTQR_OK;
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_spmm(const ctqr_sparse *A64, int32_t nslices, double alpha, const double *X, int64_t ldx,
                      double beta, double *Y, int64_t ldy, hipStream_t stream)
{
    if (!A64 || !A64->rowptr || !A64->col || !A64->val || !X || !Y || nslices < 1) return CTQR_EINVAL;
    if (ldx < A64->n || ldy < A64->m) return CTQR_EINVAL;
    return spmm_colmajor(A64->m, A64->n, nslices, A64->rowptr, A64->col, A64->val, alpha, X, ldx, beta, Y,
                         ldy, stream);
}

ctqr_status ctqr_set_progress(ctqr_progress_fn fn, void *user)
{
    std::lock_guard<std::mutex> lk(g_progress_mu);
    g_progress = fn;
    g_progress_user = user;
    return CTQR_OK;
}

ctqr_status ctqr_profile_enable(int32_t on)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (auto *v : {&g_prof, &g_prof_red}) {
        for (auto &r : *v) {
            (void)hipEventDestroy(r.a);
            (void)hipEventDestroy(r.b);
        }
        v->clear();
    }
    for (auto &r : g_phase) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    g_phase.clear();
    g_prof_on = (on & CTQR_PROFILE_UPDATE) != 0;
    g_phase_on = (on & CTQR_PROFILE_PHASES) != 0;
    return CTQR_OK;
}

ctqr_status ctqr_release(void)
{
    try {
        HIP_TRY(hipDeviceSynchronize());
        {
            std::lock_guard<std::mutex> lk(g_prof_mu);
            for (auto *v : {&g_prof, &g_prof_red}) {
                for (auto &r : *v) {
                    (void)hipEventDestroy(r.a);
                    (void)hipEventDestroy(r.b);
                }
                v->clear();
            }
            for (auto &r : g_phase) {
                (void)hipEventDestroy(r.a);
                (void)hipEventDestroy(r.b);
            }
            g_phase.clear();
            g_prof_on = g_phase_on = false;
        }
        {
            std::lock_guard<std::mutex> lk(g_progress_mu);
            g_progress = nullptr;
            g_progress_user = nullptr;
        }
        std::lock_guard<std::mutex> lk(g_flags_mu);
        for (int *p : g_flags) (void)hipHostFree(p);
        g_flags.clear();
        ++g_flags_epoch;
        return CTQR_OK;
    } catch (...) {
        return CTQR_EHIP;
    }
}

ctqr_status ctqr_profile_phases(double *ms, int64_t *count)
{
    if (!ms || !count) return CTQR_EINVAL;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    for (int p = 0; p < CTQR_NPHASES; ++p) {
        ms[p] = 0.0;
        count[p] = 0;
    }
    for (auto &r : g_phase) {
        float t = 0.f;
        HIP_TRY(hipEventSynchronize(r.b));
        HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
        ms[r.phase] += t;
        count[r.phase] += 1;
    }
    return CTQR_OK;
}

static ctqr_status profile_sum(const std::vector<ProfRec> &v, int64_t *launches, double *total_ms,
                               double *total_flops)
{
    if (!launches || !total_ms || !total_flops) return CTQR_EINVAL;
    double ms = 0.0, fl = 0.0;
    for (auto &r : v) {
        float t = 0.f;
        HIP_TRY(hipEventSynchronize(r.b));
        HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
        ms += t;
        fl += r.flops;
    }
    *launches = (int64_t)v.size();
    *total_ms = ms;
    *total_flops = fl;
    return CTQR_OK;
}

ctqr_status ctqr_profile_read_reduction(int64_t *launches, double *total_ms, double *total_flops)
{
    std::lock_guard<std::mutex> lk(g_prof_mu);
    return profile_sum(g_prof_red, launches, total_ms, total_flops);
}

ctqr_status ctqr_profile_read(int64_t *launches, double *total_ms, double *total_flops)
{
    if (!launches || !total_ms || !total_flops) return CTQR_EINVAL;
    std::lock_guard<std::mutex> lk(g_prof_mu);
    double ms = 0.0, fl = 0.0;
    for (auto &r : g_prof) {
        float t = 0.f;
        HIP_TRY(hipEventSynchronize(r.b));
        HIP_TRY(hipEventElapsedTime(&t, r.a, r.b));
        ms += t;
        fl += r.flops;
    }
    *launches = (int64_t)g_prof.size();
    *total_ms = ms;
    *total_flops = fl;
    return CTQR_OK;
}

}  // extern "C"
