// Device-wide barrier of the persistent kernels (the grid.sync() of the
// paper's Listing 1 / Listing 2), built for gfx950.
//
// Design (measured on MI355X, 256 workgroups of 512 threads):
//   * One packed arrival word per workgroup; the master workgroup
//     (workgroup 0) polls all of them, each of its waves a share of 512-word
//     chunks with eight independent loads per lane per round, and then
//     publishes a generation word that the other workgroups poll.  No
//     read-modify-write atomics: a shared counter serialises arrivals at the
//     memory side (~70 ns each).
//   * Only workgroup-scope fences.  All data that crosses workgroups is moved
//     with agent-coherent (sc1) loads and stores, so the barrier never needs
//     the agent-scope release/acquire that writes back and invalidates the
//     eight XCD-private L2 caches (3.6 us per barrier at 256 workgroups).
//   * Release: before the workgroup barrier every wave waits until its own
//     vector-memory operations have completed (vmcnt = 0).  A workgroup-scope
//     fence does not wait for them on gfx950, and s_barrier does not either,
//     so without this wait the arrival flag could reach memory before the
//     data it publishes.
//   Result: ~2.1 us per barrier at 256 workgroups, ~1.4 us at 64.
//
// Epochs: the words hold monotonically increasing epoch numbers.  A launch
// starts from the epoch the previous launch left in SYNC_EPOCH and stores its
// final epoch there before it ends, so no reset (and no memset) is needed
// between launches, including hipGraph replays.
//
// Timing: every workgroup counts the shader-clock cycles (s_memtime) it spends
// inside device barriers, from entering sync() to leaving it, and the cycles
// from its first barrier set-up to its end; at the end it stores both, and
// the number of barriers, in its own record of the SYNC_STATS area (read back
// by perks_barrier_stats).  Two scalar clock reads per barrier.
#pragma once

#include "common.hpp"

namespace perks {

// Called by the 64 lanes of wave `wave` of the `nwaves` waves that share the
// poll: returns once flags[0 .. G) of its chunks all equal e.  The flags are
// cut into chunks of 512; wave w polls chunks w, w + nwaves, ...  Each lane
// issues 8 independent flag loads per chunk, so one memory round trip covers
// a chunk, and with one chunk per wave the whole poll is one round trip (the
// waves' polls run side by side; sequential chunks would cost one round trip
// each).
__device__ __forceinline__ void wait_flags(const unsigned *flags, unsigned G, unsigned e, unsigned wave,
                                           unsigned nwaves) {
    const unsigned lane = threadIdx.x & 63;
    const unsigned first = 512u * __builtin_amdgcn_readfirstlane(wave);
    while (true) {
        bool ok = true;
        for (unsigned base = first; base < G; base += 512 * nwaves) {
            // lanes past the last workgroup load its flag again (no branch,
            // so the eight loads stay in flight together) and ignore it
            unsigned v[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) v[u] = ld_coh(flags + min(base + 64u * u + lane, G - 1));
#pragma unroll
            for (int u = 0; u < 8; ++u) ok = ok & ((base + 64u * u + lane >= G) | (v[u] == e));
        }
        if (__all(ok)) return;
        __builtin_amdgcn_s_sleep(1);
    }
}

// Waits until every vector-memory load and store this wave has issued has
// completed (s_waitcnt vmcnt(0); expcnt and lgkmcnt left at their maxima).
// Every wave of a workgroup calls it before the workgroup barrier that
// precedes the arrival-flag store: the data stores then precede the flag.
__device__ __forceinline__ void wait_own_stores() {
    __builtin_amdgcn_s_waitcnt(0x0F70);
}

// Per-workgroup barrier clock (wave-uniform values, scalar registers).
struct BarrierClock {
    unsigned long long begin, wait;
    unsigned count;

    static __device__ __forceinline__ unsigned long long now() { return __builtin_amdgcn_s_memtime(); }
    __device__ __forceinline__ void start() {
        begin = now();
        wait = 0;
        count = 0;
    }
    __device__ __forceinline__ void add(unsigned long long t0) {
        wait += now() - t0;
        ++count;
    }
    // Stores {wait, total, count} in this workgroup's record.
    __device__ __forceinline__ void publish(unsigned *ws) const {
        if (threadIdx.x == 0) {
            unsigned long long *rec = (unsigned long long *)(ws + SYNC_STATS) + SYNC_STATS_WORDS * blockIdx.x;
            const unsigned long long total = now() - begin;
            st_coh(rec + 0, wait);
            st_coh(rec + 1, total);
            st_coh(rec + 2, (unsigned long long)count);
        }
    }
};

struct GridSync {
    unsigned *ws;
    unsigned epoch;
    BarrierClock clk;

    __device__ __forceinline__ void init(unsigned *w) {
        ws = w;
        epoch = ld_coh(ws + SYNC_EPOCH);
        clk.start();
    }

    // All threads of all workgroups call this; returns when every workgroup
    // has arrived.  Global writes made before the call with st_coh (or any
    // other write that has completed) are visible to ld_coh after it.  With
    // acquire_caches, thread 0 also invalidates this CU's L1 and its XCD's L2
    // (one agent-scope acquire per workgroup), after which ordinary cached
    // loads see every st_coh store made before the barrier; that lets a
    // workgroup gather data written by others through the caches.
    template <bool acquire_caches = false>
    __device__ __forceinline__ void sync() {
        const unsigned long long t0 = BarrierClock::now();
        const unsigned e = ++epoch;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        wait_own_stores();
        __syncthreads();
        if (threadIdx.x == 0) st_coh(ws + SYNC_FLAGS + blockIdx.x, e);
        if (blockIdx.x == 0) {
            // every wave polls its chunks; the workgroup barrier joins them
            wait_flags(ws + SYNC_FLAGS, gridDim.x, e, threadIdx.x >> 6, blockDim.x >> 6);
            __syncthreads();
            if (threadIdx.x == 0) st_coh(ws + SYNC_GEN, e);
        } else if (threadIdx.x == 0) {
            while (ld_coh(ws + SYNC_GEN) != e) __builtin_amdgcn_s_sleep(1);
        }
        if (acquire_caches && threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        clk.add(t0);
    }

    // Called once by every workgroup after its last sync(): records the epoch
    // for the next launch and this workgroup's barrier clock.  Only workgroup
    // 0 writes the epoch; every workgroup has read the start epoch before the
    // first sync(), which precedes this write.
    __device__ __forceinline__ void finish() {
        if (blockIdx.x == 0 && threadIdx.x == 0) st_coh(ws + SYNC_EPOCH, epoch);
        clk.publish(ws);
    }
};

// Barrier over a group of `size` consecutive workgroups of the grid, the
// member of rank r being workgroup first + r; the same master-gather scheme as
// GridSync, with the group's own generation word.  A group of one workgroup
// synchronises with __syncthreads() alone.  Epochs start from `epoch0`, which
// every group of a launch shares (the launch's start epoch): a flag or
// generation word left over from an earlier launch holds an epoch <= epoch0,
// so it can never match.
struct GroupSync {
    unsigned *flags;   // flags of the group's workgroups, indexed by rank
    unsigned *gen;     // the group's generation word
    unsigned epoch;
    int rank, size;
    BarrierClock *clk; // the workgroup's barrier clock (shared by the groups it joins)

    __device__ __forceinline__ void init(unsigned *ws, int first, int group, int r, int n, unsigned epoch0,
                                         BarrierClock *c) {
        flags = ws + SYNC_FLAGS + first;
        gen = ws + SYNC_GROUP_GEN + group * SYNC_GROUP_STRIDE;
        rank = r;
        size = n;
        epoch = epoch0;
        clk = c;
    }
    // The whole grid as one group, epochs continuing from the last launch.
    __device__ __forceinline__ void init_grid(unsigned *ws, BarrierClock *c) {
        flags = ws + SYNC_FLAGS;
        gen = ws + SYNC_GEN;
        rank = blockIdx.x;
        size = gridDim.x;
        epoch = ld_coh(ws + SYNC_EPOCH);
        clk = c;
    }

    template <bool acquire_caches = false>
    __device__ __forceinline__ void sync() {
        if (size == 1) {
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
            __syncthreads();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
            return;
        }
        const unsigned long long t0 = BarrierClock::now();
        const unsigned e = ++epoch;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        wait_own_stores();
        __syncthreads();
        if (threadIdx.x == 0) st_coh(flags + rank, e);
        if (rank == 0) {
            wait_flags(flags, (unsigned)size, e, threadIdx.x >> 6, blockDim.x >> 6);
            __syncthreads();
            if (threadIdx.x == 0) st_coh(gen, e);
        } else if (threadIdx.x == 0) {
            while (ld_coh(gen) != e) __builtin_amdgcn_s_sleep(1);
        }
        if (acquire_caches && threadIdx.x == 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        __syncthreads();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup");
        clk->add(t0);
    }
};

}  // namespace perks
