// Internal helpers shared by the gfx950 kernels of libctqr.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include "../../include/ctqr.h"

typedef float floatx4 __attribute__((ext_vector_type(4)));
typedef float floatx16 __attribute__((ext_vector_type(16)));
typedef double doublex2 __attribute__((ext_vector_type(2)));
typedef double doublex4 __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));

#define CTQR_WAVE 64

// Host-side: return CTQR_EHIP from the enclosing function if a HIP call fails.
#define HIP_TRY(expr)                                   \
    do {                                                \
        hipError_t e_ = (expr);                         \
        if (e_ != hipSuccess) {                         \
            ctqr_last_hip_error(e_, #expr, __FILE__, __LINE__); \
            return CTQR_EHIP;                           \
        }                                               \
    } while (0)

// Launch with hipLaunchKernelGGL and check the launch status.
#define LAUNCH_TRY(kernel, grid, block, shmem, stream, ...)                    \
    do {                                                                      \
        hipLaunchKernelGGL(kernel, grid, block, shmem, stream, __VA_ARGS__); \
        HIP_TRY(hipGetLastError());                                           \
    } while (0)

void ctqr_last_hip_error(hipError_t e, const char *what, const char *file, int line);

// ---------------------------------------------------------------------------
// Device-side numerical events go into the caller's ctqr_info.  The first
// event wins (atomicCAS on status) so a later, derived event does not hide it.
// ---------------------------------------------------------------------------
__device__ inline void info_event(ctqr_info *info, int code, int col)
{
    if (!info) return;
    if (atomicCAS(&info->status, 0, code) == 0 && col >= 0) info->first_bad_col = col;
}

// ---------------------------------------------------------------------------
// Grid-wide barrier for cooperative launches (all workgroups co-resident).
// Arrival is a two-level tree: each workgroup bumps the counter of its group
// of GB_GROUP workgroups; the last arriver of a group bumps the root counter;
// the last group releases everyone by publishing the new generation, which
// the workgroups poll.  No address sees more than GB_GROUP atomics per
// barrier.  `bar` points at GB_WORDS zeroed words owned by this launch;
// `epoch` counts the barriers passed.
//
// No cache-maintenance fences: data exchanged across workgroups must be
// written with store_coherent and read with load_coherent (agent-scope
// atomics, performed at the device-coherent level past the per-XCD L2s).
// Every thread waits for its own stores to complete before the workgroup
// arrives, and the counters and the generation word are themselves atomics,
// so a workgroup that sees the new generation sees every store made before
// any arrival.
//
// The wait is bounded: after ~2^26 polls it records CTQR_BARRIER_TIMEOUT and
// lets the workgroup continue, so every wave exits.  Returns false on a
// time-out.
// ---------------------------------------------------------------------------
#define GB_GROUP 16
#define GB_LINE 32                       /* words per counter (128-byte lines) */
#define GB_MAX_GROUPS 64
#define GB_WORDS (GB_LINE * (GB_MAX_GROUPS + 2))

__device__ inline bool grid_barrier(unsigned *bar, unsigned &epoch, ctqr_info *info)
{
    __builtin_amdgcn_s_waitcnt(0);          // this thread's stores have completed
    __syncthreads();
    ++epoch;
    __shared__ int timed_out;
    if (threadIdx.x == 0) {
        timed_out = 0;
        const unsigned G = gridDim.x, g = blockIdx.x / GB_GROUP;
        const unsigned ngroups = (G + GB_GROUP - 1) / GB_GROUP;
        const unsigned gsize = min((unsigned)GB_GROUP, G - g * GB_GROUP);
        unsigned old = __hip_atomic_fetch_add(&bar[GB_LINE * (1 + g)], 1u, __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_AGENT);
        if (old == epoch * gsize - 1) {
            unsigned o2 = __hip_atomic_fetch_add(&bar[GB_LINE * (1 + GB_MAX_GROUPS)], 1u, __ATOMIC_RELAXED,
                                                 __HIP_MEMORY_SCOPE_AGENT);
            if (o2 == epoch * ngroups - 1)
                __hip_atomic_store(&bar[0], epoch, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
        unsigned polls = 0;
        while (__hip_atomic_load(&bar[0], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
            __builtin_amdgcn_s_sleep(1);
            if (++polls > (1u << 26)) {
                timed_out = 1;
                info_event(info, CTQR_BARRIER_TIMEOUT, -1);
                break;
            }
        }
    }
    __atomic_signal_fence(__ATOMIC_SEQ_CST);   // no compiler motion across the wait
    __syncthreads();
    return !timed_out;
}

// Agent-scope coherent store/load of a double, for data exchanged through
// grid_barrier.
__device__ inline void store_coherent(double *p, double v)
{
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline double load_coherent(const double *p)
{
    return __hip_atomic_load(const_cast<double *>(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

template <typename T> struct dtype_of;
template <> struct dtype_of<float> { static constexpr int value = CTQR_F32; };
template <> struct dtype_of<double> { static constexpr int value = CTQR_F64; };

static inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
