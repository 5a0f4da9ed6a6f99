// Shared host/device helpers of libperks: error reporting, scratch memory,
// coherent loads/stores for data that crosses workgroups, DPP lane shifts.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <type_traits>
#include <utility>

#include "../../include/perks.h"

namespace perks {

// ---------------------------------------------------------------------------
// Error reporting: a thread-local detail string behind perks_last_error().
int set_error(int code, const char *fmt, ...);
const char *last_error();

#define PERKS_HIP_TRY(expr)                                                              \
    do {                                                                                 \
        hipError_t e_ = (expr);                                                          \
        if (e_ != hipSuccess)                                                            \
            return ::perks::set_error(PERKS_E_HIP, "%s failed: %s (%s:%d)", #expr,       \
                                      hipGetErrorString(e_), __FILE__, __LINE__);        \
    } while (0)

// ---------------------------------------------------------------------------
// Library-owned scratch memory, one growable buffer per (device, slot).
// Growing frees the old buffer (which synchronises the device).
enum ScratchSlot {
    SLOT_SYNC = 0,      // barrier words (kept zero-initialised)
    SLOT_FACES,         // stencil halo faces (raw values, barrier mode)
    SLOT_FACES_LL,      // stencil halo faces (epoch-tagged words, point-to-point mode)
    SLOT_PINGPONG,      // per-step baseline's second grid
    SLOT_CG_VEC,        // CG work vectors
    SLOT_CG_PART,       // CG partition table / partial sums
    SLOT_NN,            // network activations, gradients, packed weights
    SLOT_FCG,           // flexible-CG work vectors
    SLOT_WIDE,          // second grid buffer of the radius-2..4 persistent stencils
    SLOT_NN_PAIRS,      // partial sums of training-pair formation
    SLOT_COUNT
};
// Returns a device pointer of at least `bytes`, or nullptr (error already set).
void *scratch(int slot, size_t bytes);

// Barrier workspace layout (32-bit words).  Flags are packed: one word per
// workgroup, written by that workgroup only.
constexpr int SYNC_GEN = 0;           // generation word released by the master
constexpr int SYNC_EPOCH = 64;        // barrier epoch carried from one launch to the next
constexpr int SYNC_LL_EPOCH = 96;     // LL face epoch carried from one launch to the next
constexpr int SYNC_AUX = 128;         // small device-side results (CG scalars, ...)
constexpr int SYNC_FLAGS = 1024;      // flags[wg]
constexpr int SYNC_MAX_WGS = 8192;
constexpr int SYNC_GROUP_GEN = SYNC_FLAGS + SYNC_MAX_WGS;   // generation word of workgroup group j
constexpr int SYNC_GROUP_STRIDE = 16;                      // at SYNC_GROUP_GEN + j * stride (own 64 B)
// Barrier clock records, one per workgroup of the last persistent launch:
// SYNC_STATS_WORDS 64-bit words each, {cycles waiting in barriers, cycles
// from the first barrier set-up to the end, barriers taken, unused}.
constexpr int SYNC_STATS = SYNC_GROUP_GEN + SYNC_MAX_WGS * SYNC_GROUP_STRIDE;
constexpr int SYNC_STATS_WORDS = 4;
constexpr size_t SYNC_BYTES = (SYNC_STATS + (size_t)SYNC_MAX_WGS * SYNC_STATS_WORDS * 2) * 4 + 4096;

struct DeviceFacts {
    int device = -1;
    int cus = 0;
    int lds_per_cu = 0;
    int regs_per_cu = 0;
    int l2 = 0;
    size_t hbm = 0;
    char arch[64] = {0};
};
int device_facts(DeviceFacts *out);

// Cooperative launch of a persistent kernel taking one by-value parameter
// struct; maps a too-large grid to PERKS_E_NOTCORESIDENT.  Records the grid
// size as the current device's last persistent launch (for its barrier clock
// records).
int launch_coop(const void *fn, int wgs, int threads, void *params, hipStream_t st);
// Records `wgs` and its barrier words `ws` (NULL: the library's shared ones)
// as the current device's last persistent launch (launches that do not go
// through launch_coop).
void note_persistent_launch(int wgs, unsigned *ws);
// Drops that record if its barrier words are `ws` (about to be freed).
void forget_persistent_launch(unsigned *ws);
// Averages the barrier clock records of the first G workgroups in the barrier
// words `ws` (NULL: the shared ones); synchronises `st` (see
// perks_barrier_stats).
int read_barrier_stats(int G, unsigned *ws, hipStream_t st, perks_barrier_stats_t *out);

}  // namespace perks

// ---------------------------------------------------------------------------
// Device helpers.
#define PERKS_AGENT __HIP_MEMORY_SCOPE_AGENT

namespace perks {

// Global-memory pointers.  Pointers held in structures that kernels load at
// run time, or laundered through opaque(), are generic to the compiler, and
// every access through a generic pointer is a flat instruction: a 64-bit
// address per lane, and counted in lgkmcnt as well as vmcnt, so that each
// wait for an LDS or scalar load also waits for every flat load in flight.
// Pointer fields typed gmem<T> * keep the global address space: accesses are
// global_* instructions with a uniform base in scalar registers and a 32-bit
// lane offset, counted by vmcnt alone.  The casts below emit no instruction.
template <typename T>
using gmem = __attribute__((address_space(1))) T;
template <typename T>
__host__ __device__ __forceinline__ gmem<T> *to_global(T *p) {
    return (gmem<T> *)p;
}

// Loads and stores of data produced or consumed by another workgroup.  They
// are relaxed agent-scope atomics: the compiler emits them with the sc1 cache
// policy, which keeps them coherent across the eight XCD-private L2 caches
// without a device-wide cache write-back or invalidate.
template <typename T>
__device__ __forceinline__ T ld_coh(const gmem<T> *p) {
    return __hip_atomic_load(const_cast<gmem<T> *>(p), __ATOMIC_RELAXED, PERKS_AGENT);
}
template <typename T>
__device__ __forceinline__ void st_coh(gmem<T> *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, PERKS_AGENT);
}
template <typename T>
__device__ __forceinline__ T ld_coh(const T *p) {
    return ld_coh<T>((const gmem<T> *)p);
}
template <typename T>
__device__ __forceinline__ void st_coh(T *p, T v) {
    st_coh<T>((gmem<T> *)p, v);
}

// Lane shifts across the 64-lane wavefront with DPP wave_shr:1 / wave_shl:1.
// shr: lane l receives lane l-1's value; lane 0 receives `fill` (lane 0's).
// shl: lane l receives lane l+1's value; lane 63 receives `fill` (lane 63's).
// With bound_ctrl off, a lane whose source is outside the wave keeps the
// "old" operand, which is how the halo value enters the edge lane.
constexpr int DPP_WAVE_SHL1 = 0x130;
constexpr int DPP_WAVE_SHR1 = 0x138;

template <int CTRL>
__device__ __forceinline__ float dpp_move(float src, float fill) {
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(fill), __float_as_int(src),
                                                      CTRL, 0xf, 0xf, false));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move(double src, double fill) {
    long long s = __double_as_longlong(src), f = __double_as_longlong(fill);
    int lo = __builtin_amdgcn_update_dpp((int)f, (int)s, CTRL, 0xf, 0xf, false);
    int hi = __builtin_amdgcn_update_dpp((int)(f >> 32), (int)(s >> 32), CTRL, 0xf, 0xf, false);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <typename T>
__device__ __forceinline__ T from_west(T v, T fill) { return dpp_move<DPP_WAVE_SHR1>(v, fill); }
template <typename T>
__device__ __forceinline__ T from_east(T v, T fill) { return dpp_move<DPP_WAVE_SHL1>(v, fill); }

// The same shifts where the edge lane's result is never used: it reads 0
// (bound_ctrl), so the value need not be copied into the destination first
// (one instruction per 32 bits instead of two).
template <int CTRL>
__device__ __forceinline__ float dpp_move0(float src) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(src), CTRL, 0xf, 0xf, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp_move0(double src) {
    long long s = __double_as_longlong(src);
    int lo = __builtin_amdgcn_mov_dpp((int)s, CTRL, 0xf, 0xf, true);
    int hi = __builtin_amdgcn_mov_dpp((int)(s >> 32), CTRL, 0xf, 0xf, true);
    return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}
template <typename T>
__device__ __forceinline__ T from_west0(T v) { return dpp_move0<DPP_WAVE_SHR1>(v); }
template <typename T>
__device__ __forceinline__ T from_east0(T v) { return dpp_move0<DPP_WAVE_SHL1>(v); }

// a*b+c with one rounding in the operands' own precision (__builtin_fma
// alone would widen float operands to double and round twice).
__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// a*b+c (one rounding) in the three-address VOP3 form.  The compiler's own
// FMA is the two-address v_fmac whose result must stay in the accumulator's
// register; when a new grid value must replace its old value in place (the
// register cache), the untied form lets the result take the old value's
// register instead of costing a copy per cell and a second register set.
__device__ __forceinline__ double fma_untied(double a, double b, double c) {
    double r;
    asm("v_fma_f64 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}
__device__ __forceinline__ float fma_untied(float a, float b, float c) {
    float r;
    asm("v_fma_f32 %0, %1, %2, %3" : "=v"(r) : "v"(a), "v"(b), "v"(c));
    return r;
}

// Hides a uniform pointer's value from the optimiser for one use site.  The
// step loops re-derive their face-buffer addresses from laundered bases every
// step; otherwise loop-invariant code motion keeps dozens of per-lane 64-bit
// addresses alive across the whole time loop, in the same registers that
// should hold the cached domain.  P is a pointer type (any address space).
template <typename P>
__device__ __forceinline__ P opaque(P p) {
    const unsigned long long a = (unsigned long long)p;
    unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)a);
    unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(a >> 32));
    asm volatile("" : "+s"(lo), "+s"(hi));
    return (P)(((unsigned long long)hi << 32) | lo);
}

// Ties the values to this point of the program: the compiler waits here for
// the loads that produce them, and later uses no longer refer to the loads.
// (vmcnt counts loads and stores alike, so a wait the compiler places after a
// step's stores would also wait for every one of them.)
template <typename T, int N>
__device__ __forceinline__ void settle(T (&a)[N]) {
#pragma unroll
    for (int i = 0; i < N; ++i) asm volatile("" : "+v"(a[i]));
}

// Calls f(integral_constant<int, I>) for I = B .. E-1 (a compile-time loop:
// every register-array index stays constant, whatever the unroller decides).
template <int B, int E, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (B < E) {
        f(std::integral_constant<int, B>{});
        static_for<B + 1, E>(f);
    }
}

// Keeps the compiler from moving memory operations across this point.  LDS
// operations of one wavefront complete in program order, so a wave that
// writes LDS and then reads it needs no hardware barrier.
__device__ __forceinline__ void compiler_fence() { __atomic_signal_fence(__ATOMIC_SEQ_CST); }

}  // namespace perks
