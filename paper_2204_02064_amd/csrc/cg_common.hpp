// Helpers shared by the persistent Krylov kernels (CG, mixed-precision CG,
// flexible CG): launch shape, wave / group / workgroup reductions with a fixed
// summation order, the fixed-order all-reduce over a group of workgroups,
// and the merge-path row split.
#pragma once

#include "common.hpp"

namespace perks {
namespace {

#ifndef PERKS_CG_WAVES
#define PERKS_CG_WAVES 16
#endif
#ifndef PERKS_CG_U
#define PERKS_CG_U 4
#endif
constexpr int CG_WAVES = PERKS_CG_WAVES;
constexpr int CG_THREADS = CG_WAVES * 64;

// Sum over the 64 lanes of a wave (butterfly; every lane gets the total).
__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Sum over groups of L lanes (L a power of two, runtime-uniform).
template <typename T>
__device__ __forceinline__ T group_sum(T v, int L) {
    for (int off = L >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    return v;
}

// Deterministic workgroup sum of up to 3 values: waves reduce, then wave 0
// adds the wave totals in wave order.  Returns the sums to thread 0 only.
template <int K>
__device__ __forceinline__ void block_sum(double (&v)[K], double *lds_red) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) lds_red[k * CG_WAVES + wave] = v[k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int w = 0; w < CG_WAVES; ++w) s += lds_red[k * CG_WAVES + w];
            v[k] = s;
        }
    }
    __syncthreads();
}

// A value every lane holds alike, moved to scalar registers.
__device__ __forceinline__ double uniform(double v) {
    const long long b = __double_as_longlong(v);
    const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)b);
    const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(b >> 32));
    return __longlong_as_double(((long long)hi << 32) | lo);
}

// Every workgroup of a group of G sums the G partials of slot `slot` in the
// same order (lanes take strided shares, then a butterfly): identical bits
// everywhere.
__device__ __forceinline__ double grid_total(const double *part, int slot, int G, double *lds_bcast) {
    if (threadIdx.x < 64) {
        double s = 0.0;
        for (int i = threadIdx.x; i < G; i += 64) s += ld_coh(part + (size_t)slot * G + i);
        s = wave_sum(s);
        if (threadIdx.x == 0) *lds_bcast = s;
    }
    __syncthreads();
    const double t = uniform(*lds_bcast);
    __syncthreads();
    return t;
}

// First row of share g when rows + nonzeros are split into G equal shares:
// the smallest i with i + rowptr[i] >= g * (n + nnz) / G (merge-path diagonal).
__device__ int merge_split(const int *rowptr, int n, int nnz, int g, int G) {
    const long long target = (long long)g * ((long long)n + nnz) / G;
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if ((long long)mid + rowptr[mid] < target) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ int pick_group(int rows, int nnz) {
    const int avg = rows > 0 ? (nnz + rows - 1) / rows : 1;
    int L = 1;
    while (L < avg && L < 64) L <<= 1;
    return L;
}

}  // namespace
}  // namespace perks
