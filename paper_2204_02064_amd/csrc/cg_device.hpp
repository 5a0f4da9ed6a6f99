// Device side of the persistent CG solvers (Sec. 2.2.2, Sec. 4.3): problem
// description, SpMV layouts, the FP64, register-resident, mixed-precision and
// batched solver bodies and their kernels.  Included by cg.hip (16 waves per
// workgroup) and by cg_reg.hip, which builds the register-resident solver
// with 8 waves per workgroup (PERKS_CG_WAVES) so that each wave has 256
// registers for its rows' vectors.  Everything is in an unnamed namespace:
// each translation unit gets its own copy, compiled for its wave count.
#pragma once

#include <algorithm>
#include <cmath>

#include "barrier.hpp"
#include "cg_common.hpp"
#include "common.hpp"

namespace perks {
namespace {

enum { PART_PQ = 0, PART_RZ = 1, PART_RR = 2, PART_BB = 3, PART_TRUE = 4, NPART = 5 };

// One CG problem and its work vectors (device pointers).  FP64 solves use
// r, z, q, p, dinv; mixed solves use r64 and the FP32 vectors.  part
// holds NPART partial sums per workgroup of the problem's group; result
// receives iters, status, relres, relres_true, ||b||, restarts or outer steps.
struct CgInst {
    const int *rowptr;
    const int *colind;
    const double *val;
    const double *b;
    double *x;
    double *r, *z, *q, *p, *dinv;
    float *val32;
    double *r64;
    float *r32, *z32, *q32, *p32, *d32, *dinv32;
    double *part;
    double *result;
    double *sval64;          // sliced-ELL copy of A (FP64 solver), NULL: CSR only
    float *sval32;           // sliced-ELL copy of A (mixed solver)
    int *scol;               // its column indices
    int *sperm;              // rows of each workgroup's slice in sliced-ELL order (n entries)
    double *cap_x, *cap_r;   // FP64 solver: x and r after the iterations listed in cap_iters
    const int *cap_iters;    // ascending iteration counts (device)
    int ncap;
    int spmv;                // SpMV layout requested: 0 the library's choice, 1 sliced ELL / CSR, 2 merge path
    int n;
    int nnz;
    int maxit;
    int max_outer;
    double tol;
    double update_tol;
};

// The problem description as kernels read it: through the constant address
// space (the host writes it before the launch, no kernel writes it), so that
// the compiler takes every pointer loaded from it to address global memory
// and emits global_* accesses instead of flat ones (which also count in
// lgkmcnt, making every LDS wait of the SpMV wait for the gathers too).
using CInst = const __attribute__((address_space(4))) CgInst;

// The workgroup's LDS copy of (the first entries of) its slice of A: FP64
// values for the FP64 solver, FP32 values for the mixed-precision solver.
// Each kernel references only its own pair, so each gets only that pair.
constexpr int CG_LDS_NNZ = 12032;     // 141 KiB of the 160 KiB LDS (12 B/nonzero)
constexpr int CG_LDS_NNZ32 = 18048;   // 141 KiB (8 B/nonzero)
__shared__ double cg_lval[CG_LDS_NNZ];
__shared__ int cg_lcol[CG_LDS_NNZ];
__shared__ float cg_lval32[CG_LDS_NNZ32];
__shared__ int cg_lcol32[CG_LDS_NNZ32];

template <typename T> struct LdsA;
template <> struct LdsA<double> {
    static constexpr int cap = CG_LDS_NNZ;
    static __device__ __forceinline__ double &val(int k) { return cg_lval[k]; }
    static __device__ __forceinline__ int &col(int k) { return cg_lcol[k]; }
};
template <> struct LdsA<float> {
    static constexpr int cap = CG_LDS_NNZ32;
    static __device__ __forceinline__ float &val(int k) { return cg_lval32[k]; }
    static __device__ __forceinline__ int &col(int k) { return cg_lcol32[k]; }
};

// y_i for rows [r0, r1) with L lanes per row: sum_k a_k * v(col_k) in type T,
// where v(j) is produced by `fetch`.  FROM_LDS: the rows lie wholly in the
// LDS copy of the slice (entry k at index k - kbase); otherwise A is read from
// `gval` in global memory.  Each lane group takes U rows per pass and issues
// all their loads before any use (U times the memory-level parallelism of one
// row at a time).  A row's sum is the lane-strided partial sums followed by
// the group butterfly: its rounding depends neither on U nor on where A is
// read from.
template <int U, bool FROM_LDS, typename T, typename F, typename S>
__device__ __forceinline__ void spmv_range(const int *rowptr, const int *colind, const T *gval, int r0, int r1,
                                           int L, int kbase, F fetch, S sink) {
    const int tid = threadIdx.x;
    const int gl = tid & (L - 1);
    const int rpp = CG_THREADS / L;
    for (int row0 = r0; row0 < r1; row0 += rpp * U) {
        int kb[U], ke[U];
        T s[U];
        int len = 0;
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int i = row0 + u * rpp + tid / L;
            kb[u] = 0;
            ke[u] = 0;
            s[u] = T(0);
            if (i < r1) {
                kb[u] = rowptr[i] + gl;
                ke[u] = rowptr[i + 1];
            }
            len = max(len, ke[u] - kb[u]);
        }
        for (int j = 0; j < len; j += L) {
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int k = kb[u] + j;
                if (k < ke[u]) {
                    T a;
                    int c;
                    if constexpr (FROM_LDS) {
                        a = LdsA<T>::val(k - kbase);
                        c = LdsA<T>::col(k - kbase);
                    } else {
                        a = gval[k];
                        c = colind[k];
                    }
                    s[u] = fma_t(a, fetch(c), s[u]);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const T t = group_sum(s[u], L);
            const int i = row0 + u * rpp + tid / L;
            if (i < r1 && gl == 0) sink(i, t);
        }
    }
}

// Rows [r0, rc) come from the LDS copy, rows [rc, r1) from global memory.
template <int U, typename T, typename F, typename S>
__device__ __forceinline__ void spmv_rows(const int *rowptr, const int *colind, const T *gval, int r0, int rc,
                                          int r1, int L, int kbase, F fetch, S sink) {
    spmv_range<U, true>(rowptr, colind, gval, r0, rc, L, kbase, fetch, sink);
    spmv_range<U, false>(rowptr, colind, gval, rc, r1, L, kbase, fetch, sink);
}

// First row of [r0, r1) that does not end within the first kc entries of the
// slice starting at kbase (rows before it are wholly cached).
__device__ __forceinline__ int cached_rows_end(const int *rowptr, int r0, int r1, int kbase, int kc) {
    int lo = r0, hi = r1;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (rowptr[mid + 1] - kbase <= kc) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

constexpr int CG_U = PERKS_CG_U;

__shared__ double cg_red[4 * CG_WAVES];
__shared__ double cg_bcast;

// The workgroup's share of a problem solved by a group of G workgroups, of
// which this one has rank g: rows [r0, r1) (merge-path split).
//
// Two layouts of the slice's rows:
// * sliced ELL (when padding costs at most a quarter more entries): chunks of
//   64 consecutive rows, one lane per row, the chunk's rows padded to its
//   longest row and stored entry-major (entry j of the chunk's rows is 64
//   consecutive values), built by the workgroup at kernel start in its own
//   region of the packed arrays.  Loads are coalesced, no row pointers are
//   read in the iterations, no lanes are reduced across.  Padding entries are
//   0 * x[row].  Chunks [0, cc) are also held in LDS.
// * CSR with L lanes per row otherwise (irregular row lengths): the first kc
//   nonzeros in LDS, rows [r0, rc) wholly cached.
// A row's sum is the same either way up to rounding order; its order depends
// only on the layout, which depends only on the problem and G.
constexpr int SELL_MAX_CHUNKS = 2048;
__shared__ int cg_chunk_len[SELL_MAX_CHUNKS];
__shared__ int cg_chunk_off[SELL_MAX_CHUNKS];
__shared__ int cg_flag;

struct Slice {
    int r0, r1, rc, kbase, nnz, kc, L;
    int sell, nch, cc, sbase;
    const int *perm;   // sliced-ELL row order (rows sorted by length), or NULL: natural order
    int merge;         // merge-path layout (see spmv_merge)
    int nchunks;       // merge path: chunks of MERGE_IPT items
    const int *mrow;   // merge path: first row (slice-relative) of chunk c, c = 0 .. nchunks
};

// Merge-path SpMV (Merrill and Garland's merge-based CSR SpMV, the SpMV the
// paper's CG uses, Sec. 4.3.1): the slice's row ends and nonzeros form one
// path of nrows + nnz items, cut into chunks of MERGE_IPT consecutive items,
// one chunk per thread per tile of CG_THREADS chunks.  Each chunk's start
// (row, nonzero) is found by a binary search on the merge diagonal once, at
// kernel start, and kept in memory for every later SpMV (A is static, so the
// search results are too: Sec. 4.3.2).
constexpr int MERGE_IPT = 8;

// Entries the packed arrays of one problem need for G workgroups.
__host__ __device__ inline size_t sell_capacity(int64_t nnz, int G) {
    return (size_t)(nnz + nnz / 4) + 64 * (size_t)G + 64;
}

// sval64, when given (mixed-precision solvers), also receives the FP64 values
// of the sliced-ELL layout (from p.val), for the FP64 residual replacements.
template <typename T, bool MERGE = false>
__device__ __forceinline__ Slice load_slice(CInst &p, const T *val, T *sval, int *scol, int g, int G,
                                            double *sval64 = nullptr) {
    Slice sl;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    sl.r0 = merge_split(p.rowptr, p.n, p.nnz, g, G);
    sl.r1 = merge_split(p.rowptr, p.n, p.nnz, g + 1, G);
    sl.kbase = p.rowptr[sl.r0];
    sl.nnz = p.rowptr[sl.r1] - sl.kbase;
    sl.L = pick_group(sl.r1 - sl.r0, sl.nnz);
    sl.nch = (sl.r1 - sl.r0 + 63) / 64;
    sl.sbase = (int)(sl.kbase + sl.kbase / 4) + 64 * g;
    __syncthreads();   // the previous problem of this workgroup is done with LDS
    sl.merge = MERGE && p.spmv == 2 && scol != nullptr;
    sl.nchunks = 0;
    sl.mrow = nullptr;
    // chunk lengths (longest row of each chunk), then their offsets
    sl.sell = !sl.merge && sval != nullptr && sl.nch <= SELL_MAX_CHUNKS;
    if (sl.sell) {
        for (int c = wave; c < sl.nch; c += CG_WAVES) {
            const int i = sl.r0 + 64 * c + lane;
            int len = i < sl.r1 ? p.rowptr[i + 1] - p.rowptr[i] : 0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
            if (lane == 0) cg_chunk_len[c] = len;
        }
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int c = 0; c < sl.nch; ++c) {
                cg_chunk_off[c] = acc;
                acc += 64 * cg_chunk_len[c];
            }
            cg_flag = acc <= sl.nnz + sl.nnz / 4 + 64 ? acc : -1;
        }
        __syncthreads();
        sl.sell = cg_flag >= 0;
    }
    sl.perm = nullptr;
    const int nrows = sl.r1 - sl.r0;
    if (!sl.merge && !sl.sell && sval != nullptr && p.sperm != nullptr && sl.nch <= SELL_MAX_CHUNKS &&
        nrows <= LdsA<T>::cap) {
        // Irregular rows: sliced ELL over the slice's rows sorted by length,
        // longest first (SELL-C-sigma with sigma = the slice), so that each
        // chunk's rows have nearly equal lengths.  A stable counting sort on
        // min(length, 255); its order depends only on the problem and G.
        int *key = &LdsA<T>::col(0);
        int *cnt = cg_chunk_off;   // 256 bucket counters, then starts
        for (int r = tid; r < nrows; r += CG_THREADS) {
            const int i = sl.r0 + r;
            key[r] = 255 - min(p.rowptr[i + 1] - p.rowptr[i], 255);
        }
        for (int b = tid; b < 256; b += CG_THREADS) cnt[b] = 0;
        __syncthreads();
        for (int r = tid; r < nrows; r += CG_THREADS) atomicAdd(&cnt[key[r]], 1);
        __syncthreads();
        if (wave == 0) {
            // exclusive prefix over the 256 buckets: 4 per lane, then a wave scan
            int c4[4], tot = 0;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                c4[u] = cnt[4 * lane + u];
                tot += c4[u];
            }
            int incl = tot;
#pragma unroll
            for (int off = 1; off < 64; off <<= 1) {
                const int t = __shfl_up(incl, off, 64);
                if (lane >= off) incl += t;
            }
            int run = incl - tot;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                cnt[4 * lane + u] = run;
                run += c4[u];
            }
            // stable scatter, 64 rows at a time: rank among equal keys from
            // ballots over the key bits
            const unsigned long long lt = (1ULL << lane) - 1ULL;
            for (int base = 0; base < nrows; base += 64) {
                const int r = base + lane;
                const int k = r < nrows ? key[r] : 256;
                unsigned long long same = __ballot(1);
#pragma unroll
                for (int bit = 0; bit < 9; ++bit) {
                    const unsigned long long m = __ballot((k >> bit) & 1);
                    same &= ((k >> bit) & 1) ? m : ~m;
                }
                const int rank = __popcll(same & lt);
                if (r < nrows) {
                    const int pos = cnt[k] + rank;
                    st_coh(p.sperm + sl.r0 + pos, sl.r0 + r);
                }
                __builtin_amdgcn_wave_barrier();
                if (r < nrows && rank == 0) cnt[k] += __popcll(same);
                __builtin_amdgcn_wave_barrier();
            }
        }
        __syncthreads();
        sl.perm = p.sperm + sl.r0;
        for (int c = wave; c < sl.nch; c += CG_WAVES) {
            const int r = 64 * c + lane;
            const int i = r < nrows ? ld_coh(sl.perm + r) : sl.r0;
            int len = r < nrows ? p.rowptr[i + 1] - p.rowptr[i] : 0;
#pragma unroll
            for (int off = 32; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
            if (lane == 0) cg_chunk_len[c] = len;
        }
        __syncthreads();
        if (tid == 0) {
            int acc = 0;
            for (int c = 0; c < sl.nch; ++c) {
                cg_chunk_off[c] = acc;
                acc += 64 * cg_chunk_len[c];
            }
            cg_flag = acc <= sl.nnz + sl.nnz / 4 + 64 ? acc : -1;
        }
        __syncthreads();
        sl.sell = cg_flag >= 0;
        if (!sl.sell) sl.perm = nullptr;
    }
    if (sl.sell) {
        // cached chunks: a prefix whose entries fit in LDS
        int cc = 0;
        while (cc < sl.nch && cg_chunk_off[cc] + 64 * cg_chunk_len[cc] <= LdsA<T>::cap) ++cc;
        sl.cc = cc;
        for (int c = wave; c < sl.nch; c += CG_WAVES) {
            const int r = 64 * c + lane;
            const int i = r < nrows ? (sl.perm ? ld_coh(sl.perm + r) : sl.r0 + r) : sl.r1;
            const int len = cg_chunk_len[c], off = cg_chunk_off[c];
            const int kb = i < sl.r1 ? p.rowptr[i] : 0;
            const int kn = i < sl.r1 ? p.rowptr[i + 1] - kb : 0;
            const int self = i < sl.r1 ? i : sl.r0;
            for (int j = 0; j < len; ++j) {
                const T a = j < kn ? val[kb + j] : T(0);
                const int cidx = j < kn ? p.colind[kb + j] : self;
                const int e = off + j * 64 + lane;
                sval[sl.sbase + e] = a;
                scol[sl.sbase + e] = cidx;
                if (sval64) sval64[sl.sbase + e] = j < kn ? p.val[kb + j] : 0.0;
                if (c < cc) {
                    LdsA<T>::val(e) = a;
                    LdsA<T>::col(e) = cidx;
                }
            }
        }
        sl.kc = 0;
        sl.rc = sl.r0;
    } else {
        sl.cc = 0;
        sl.kc = min(sl.nnz, LdsA<T>::cap);
        for (int k = tid; k < sl.kc; k += CG_THREADS) {
            LdsA<T>::val(k) = val[sl.kbase + k];
            LdsA<T>::col(k) = p.colind[sl.kbase + k];
        }
        sl.rc = cached_rows_end(p.rowptr, sl.r0, sl.r1, sl.kbase, sl.kc);
        if (sl.merge) {
            // chunk c starts on merge diagonal d = c * MERGE_IPT: its first row is
            // the number of rows whose end comes before item d, the smallest i
            // with end(i) + i >= d (end(i) = rowptr[r0 + i + 1] - kbase).  Stored
            // in this problem's otherwise unused sliced-ELL index array, at an
            // offset no other workgroup's chunks reach.
            const long long lw = (long long)nrows + sl.nnz;
            sl.nchunks = (int)((lw + MERGE_IPT - 1) / MERGE_IPT);
            int *mrow = scol + (size_t)(((long long)sl.r0 + sl.kbase) / MERGE_IPT) + 2 * (size_t)g;
            for (int c = tid; c <= sl.nchunks; c += CG_THREADS) {
                const long long d = std::min((long long)c * MERGE_IPT, lw);
                int lo = 0, hi = nrows;
                while (lo < hi) {
                    const int mid = (lo + hi) >> 1;
                    if ((long long)(p.rowptr[sl.r0 + mid + 1] - sl.kbase) + mid < d) lo = mid + 1;
                    else hi = mid;
                }
                mrow[c] = lo;
            }
            sl.mrow = mrow;
        }
    }
    __syncthreads();   // also publishes the packed arrays within the workgroup
    return sl;
}

#ifndef PERKS_SELL_U
#define PERKS_SELL_U 4
#endif
// Entries of a row whose loads and gathers are issued before their products.
constexpr int SELL_U = PERKS_SELL_U;

// Row sum of this lane's row in sliced-ELL chunk c: sum_j a_j * v(col_j),
// entries in CSR order, SELL_U entries' loads and gathers issued before their
// products; FROM_LDS: the chunk is held in LDS.
template <bool FROM_LDS, typename T, typename F>
__device__ __forceinline__ T sell_chunk(const Slice &sl, const T *sval, const int *scol, int c, int lane, F fetch) {
    const int len = cg_chunk_len[c], off = cg_chunk_off[c];
    T acc = T(0);
    int j = 0;
#pragma unroll 1
    for (; j + SELL_U <= len; j += SELL_U) {
        T a[SELL_U];
        int cidx[SELL_U];
#pragma unroll
        for (int u = 0; u < SELL_U; ++u) {
            const int e = off + (j + u) * 64 + lane;
            if constexpr (FROM_LDS) {
                a[u] = LdsA<T>::val(e);
                cidx[u] = LdsA<T>::col(e);
            } else {
                a[u] = sval[sl.sbase + e];
                cidx[u] = scol[sl.sbase + e];
            }
        }
        T xv[SELL_U];
#pragma unroll
        for (int u = 0; u < SELL_U; ++u) xv[u] = fetch(cidx[u]);
#pragma unroll
        for (int u = 0; u < SELL_U; ++u) acc = fma_t(a[u], xv[u], acc);
    }
#pragma unroll 1
    for (; j < len; ++j) {
        const int e = off + j * 64 + lane;
        T a;
        int cidx;
        if constexpr (FROM_LDS) {
            a = LdsA<T>::val(e);
            cidx = LdsA<T>::col(e);
        } else {
            a = sval[sl.sbase + e];
            cidx = scol[sl.sbase + e];
        }
        acc = fma_t(a, fetch(cidx), acc);
    }
    return acc;
}

// Register-resident own rows.  The memory-resident solver runs CG_REF_WAVES
// (16) waves per workgroup; in the natural-order sliced-ELL layout its wave w
// computes chunks c = w + 16 j, i.e. thread t = 64 w + lane computes rows
// r0 + t + 1024 j (j = 0, 1, ...), the same rows, in the same order, that its
// own-row loops give it.  The register-resident solver reproduces that
// arithmetic with CG_WAVES waves: each thread plays VT = 16 / CG_WAVES of
// those "reference threads" (virtual wave v = wave + CG_WAVES h, h < VT),
// keeps one partial sum per reference thread and adds the 16 virtual waves'
// sums in the reference order, so both solvers give the same bits.  With at
// most CG_RV rows per reference thread, the vector entries of a thread's
// VT * CG_RV rows stay in registers across iterations (the paper also caches
// the residual and the intermediate results next to A, Sec. 4.3.2).
#ifndef PERKS_CG_CHUNK_FENCE
#define PERKS_CG_CHUNK_FENCE 1
#endif
#ifndef PERKS_CG_PAIR
#define PERKS_CG_PAIR 0
#endif
constexpr int CG_REF_WAVES = 16;
constexpr int CG_REF_THREADS = CG_REF_WAVES * 64;
#ifndef PERKS_CG_RV
#define PERKS_CG_RV 10
#endif
constexpr int CG_RV = PERKS_CG_RV;
constexpr int CG_VT = CG_REF_WAVES / CG_WAVES;
static_assert(CG_REF_WAVES % CG_WAVES == 0, "the wave count must divide the reference wave count");
__shared__ double cg_red_ref[4 * CG_REF_WAVES];

// sell_chunk with the entries taken in groups of U whose loads and gathers
// are all issued before their products, the last group predicated (the
// chunk's length is wave-uniform): one memory round trip per U entries and
// no one-entry tail.  Same products, same order, same sum.
#ifndef PERKS_CG_REG_U
#define PERKS_CG_REG_U 8
#endif
template <bool FROM_LDS, typename T, typename F>
__device__ __forceinline__ T sell_chunk_grouped(const Slice &sl, const T *sval, const int *scol, int c, int lane,
                                                F fetch) {
    constexpr int U = PERKS_CG_REG_U;
    const int len = cg_chunk_len[c], off = cg_chunk_off[c];
    T acc = T(0);
#pragma unroll 1
    for (int j = 0; j < len; j += U) {
        T a[U], xv[U];
        int cidx[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            a[u] = T(0);
            cidx[u] = 0;
            if (j + u < len) {
                const int e = off + (j + u) * 64 + lane;
                if constexpr (FROM_LDS) {
                    a[u] = LdsA<T>::val(e);
                    cidx[u] = LdsA<T>::col(e);
                } else {
                    a[u] = sval[sl.sbase + e];
                    cidx[u] = scol[sl.sbase + e];
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) xv[u] = j + u < len ? fetch(cidx[u]) : T(0);
#pragma unroll
        for (int u = 0; u < U; ++u)
            if (j + u < len) acc = fma_t(a[u], xv[u], acc);
    }
    return acc;
}

// Two chunks' sums at once (sell_chunk_grouped of each, their groups
// interleaved): twice the loads in flight per round trip.
template <bool FROM_LDS, typename T, typename F>
__device__ __forceinline__ void sell_chunk_pair(const Slice &sl, const T *sval, const int *scol, int c0, int c1,
                                                int lane, F fetch, T &acc0, T &acc1) {
    constexpr int U = PERKS_CG_REG_U;
    const int len0 = cg_chunk_len[c0], off0 = cg_chunk_off[c0];
    const int len1 = cg_chunk_len[c1], off1 = cg_chunk_off[c1];
    const int len = max(len0, len1);
    acc0 = T(0);
    acc1 = T(0);
#pragma unroll 1
    for (int j = 0; j < len; j += U) {
        T a[2][U], xv[2][U];
        int cidx[2][U];
#pragma unroll
        for (int q = 0; q < 2; ++q) {
            const int lq = q ? len1 : len0, oq = q ? off1 : off0;
#pragma unroll
            for (int u = 0; u < U; ++u) {
                a[q][u] = T(0);
                cidx[q][u] = 0;
                if (j + u < lq) {
                    const int e = oq + (j + u) * 64 + lane;
                    if constexpr (FROM_LDS) {
                        a[q][u] = LdsA<T>::val(e);
                        cidx[q][u] = LdsA<T>::col(e);
                    } else {
                        a[q][u] = sval[sl.sbase + e];
                        cidx[q][u] = scol[sl.sbase + e];
                    }
                }
            }
        }
#pragma unroll
        for (int q = 0; q < 2; ++q)
#pragma unroll
            for (int u = 0; u < U; ++u) xv[q][u] = j + u < (q ? len1 : len0) ? fetch(cidx[q][u]) : T(0);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (j + u < len0) acc0 = fma_t(a[0][u], xv[0][u], acc0);
            if (j + u < len1) acc1 = fma_t(a[1][u], xv[1][u], acc1);
        }
    }
}

// A per-lane value hidden from the optimiser at this point: addresses derived
// from it after the call cannot be hoisted above it (out of the solver's
// iteration loop, where one per row and vector would stay live in registers).
__device__ __forceinline__ int launder_v(int v) {
    asm volatile("" : "+v"(v));
    return v;
}

// Row m = h * CG_RV + j of this thread: reference thread 64 (wave + CG_WAVES h)
// + lane, its j-th row.
__device__ __forceinline__ int reg_row(int r0, int wave, int lane, int m) {
    const int h = m / CG_RV, j = m % CG_RV;
    return r0 + 64 * (wave + CG_WAVES * h) + lane + CG_REF_THREADS * j;
}

// The SpMV of spmv_slice in register-row order: sink(m, i, s) for the
// thread's row m (a compile-time constant), rows of one reference thread in
// ascending j.
template <typename T, typename F, typename S>
__device__ __forceinline__ void spmv_sell_reg(const Slice &sl, const T *sval, const int *scol, F fetch, S sink) {
    const int lane = launder_v(threadIdx.x & 63), wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
#if PERKS_CG_PAIR
    // rows m and m + 1 (two consecutive rows of one reference thread) together
    static_for<0, CG_VT * CG_RV / 2>([&](auto pc) {
        constexpr int m0 = 2 * decltype(pc)::value, m1 = m0 + 1;
        const int c0 = wave + CG_WAVES * (m0 / CG_RV) + CG_REF_WAVES * (m0 % CG_RV);
        const int c1 = wave + CG_WAVES * (m1 / CG_RV) + CG_REF_WAVES * (m1 % CG_RV);
        if (c1 < sl.nch && (c0 < sl.cc) == (c1 < sl.cc)) {
            T s0, s1;
            if (c0 < sl.cc) sell_chunk_pair<true>(sl, sval, scol, c0, c1, lane, fetch, s0, s1);
            else sell_chunk_pair<false>(sl, sval, scol, c0, c1, lane, fetch, s0, s1);
            const int i0 = sl.r0 + 64 * c0 + lane, i1 = sl.r0 + 64 * c1 + lane;
            if (i0 < sl.r1) sink(std::integral_constant<int, m0>{}, i0, s0);
            if (i1 < sl.r1) sink(std::integral_constant<int, m1>{}, i1, s1);
        } else {
            if (c0 < sl.nch) {
                const int i = sl.r0 + 64 * c0 + lane;
                const T acc = c0 < sl.cc ? sell_chunk_grouped<true>(sl, sval, scol, c0, lane, fetch)
                                         : sell_chunk_grouped<false>(sl, sval, scol, c0, lane, fetch);
                if (i < sl.r1) sink(std::integral_constant<int, m0>{}, i, acc);
            }
            if (c1 < sl.nch) {
                const int i = sl.r0 + 64 * c1 + lane;
                const T acc = c1 < sl.cc ? sell_chunk_grouped<true>(sl, sval, scol, c1, lane, fetch)
                                         : sell_chunk_grouped<false>(sl, sval, scol, c1, lane, fetch);
                if (i < sl.r1) sink(std::integral_constant<int, m1>{}, i, acc);
            }
        }
#if PERKS_CG_CHUNK_FENCE
        __builtin_amdgcn_sched_barrier(0);
#endif
    });
#else
    static_for<0, CG_VT * CG_RV>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        const int c = wave + CG_WAVES * (m / CG_RV) + CG_REF_WAVES * (m % CG_RV);
        if (c < sl.nch) {
            const int i = sl.r0 + 64 * c + lane;
            const T acc = c < sl.cc ? sell_chunk_grouped<true>(sl, sval, scol, c, lane, fetch)
                                    : sell_chunk_grouped<false>(sl, sval, scol, c, lane, fetch);
            if (i < sl.r1) sink(mc, i, acc);
        }
#if PERKS_CG_CHUNK_FENCE
        // one chunk at a time: without the fence the scheduler may overlap the
        // chunks' loads and run out of registers
        __builtin_amdgcn_sched_barrier(0);
#endif
    });
#endif
}

// block_sum of the reference solver from per-reference-thread partials
// v[h][k]: wave sums, then the 16 virtual waves' sums in order (thread 0).
template <int K>
__device__ __forceinline__ void block_sum_ref(double (&v)[CG_VT][K]) {
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int h = 0; h < CG_VT; ++h)
#pragma unroll
        for (int k = 0; k < K; ++k) v[h][k] = wave_sum(v[h][k]);
    if (lane == 0) {
#pragma unroll
        for (int h = 0; h < CG_VT; ++h)
#pragma unroll
            for (int k = 0; k < K; ++k) cg_red_ref[k * CG_REF_WAVES + wave + CG_WAVES * h] = v[h][k];
    }
    __syncthreads();
    if (threadIdx.x == 0) {
#pragma unroll
        for (int k = 0; k < K; ++k) {
            double s = 0.0;
            for (int w = 0; w < CG_REF_WAVES; ++w) s += cg_red_ref[k * CG_REF_WAVES + w];
            v[0][k] = s;
        }
    }
    __syncthreads();
}

__shared__ double cg_merge_f[CG_WAVES];
__shared__ double cg_merge_s[CG_WAVES];

// y_i for the slice's rows by the merge path.  Per tile, thread t takes chunk
// c = tile + t: it loads the chunk's nonzeros (at most MERGE_IPT; from the LDS
// copy of A for entries below kc) and their gathers at once, then walks the
// chunk's items in path order: a nonzero adds a * v(col) to the running sum,
// a row end completes that row.  A row that began in an earlier chunk gets
// that chunk's partial sum through a segmented scan over the tile's chunks in
// thread order (the carry of the chunk before the first row end, plus the
// carries of the chunks before it that completed no row) and the tile's carry
// from the tile before; rows completed inside a chunk go straight to sink.
// Every sum's order depends only on the matrix and the chunk size.
template <typename T, typename F, typename S>
__device__ __forceinline__ void spmv_merge(CInst &p, const Slice &sl, const T *val, F fetch, S sink) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int nrows = sl.r1 - sl.r0;
    const long long lw = (long long)nrows + sl.nnz;
    const int *rowend = p.rowptr + sl.r0 + 1;   // rowend[i] - kbase: end of row i within the slice
    T tile_carry = T(0);
    for (int c0 = 0; c0 < sl.nchunks; c0 += CG_THREADS) {
        const int c = c0 + tid;
        int i = 0, i1 = 0, j = 0, j1 = 0;
        if (c < sl.nchunks) {
            i = sl.mrow[c];
            i1 = sl.mrow[c + 1];
            j = (int)((long long)c * MERGE_IPT - i);
            j1 = (int)(std::min((long long)(c + 1) * MERGE_IPT, lw) - i1);
        }
        T a[MERGE_IPT], xv[MERGE_IPT];
        int cidx[MERGE_IPT];
#pragma unroll
        for (int k = 0; k < MERGE_IPT; ++k) {
            a[k] = T(0);
            cidx[k] = 0;
            const int e = j + k;
            if (e < j1) {
                if (e < sl.kc) {
                    a[k] = LdsA<T>::val(e);
                    cidx[k] = LdsA<T>::col(e);
                } else {
                    a[k] = val[sl.kbase + e];
                    cidx[k] = p.colind[sl.kbase + e];
                }
            }
        }
#pragma unroll
        for (int k = 0; k < MERGE_IPT; ++k) xv[k] = j + k < j1 ? fetch(cidx[k]) : T(0);
        T acc = T(0), first_val = T(0);
        int first_row = -1;
        int iend = i < i1 ? rowend[i] - sl.kbase : 0x7fffffff;
        auto complete = [&](int r) {
            if (first_row < 0) {
                first_row = r;
                first_val = acc;
            } else {
                sink(sl.r0 + r, acc);
            }
            acc = T(0);
        };
#pragma unroll
        for (int k = 0; k < MERGE_IPT; ++k) {
            if (j + k < j1) {
                while (i < i1 && iend <= j + k) {
                    complete(i);
                    ++i;
                    iend = i < i1 ? rowend[i] - sl.kbase : 0x7fffffff;
                }
                acc = fma_t(a[k], xv[k], acc);
            }
        }
        while (i < i1) {   // rows ending after the chunk's last nonzero
            complete(i);
            ++i;
        }
        // segmented scan of (completed a row, carry) over the tile's chunks
        bool f = first_row >= 0;
        T sc = acc;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) {
            const T su = __shfl_up(sc, off, 64);
            const int fu = __shfl_up((int)f, off, 64);
            if (lane >= off) {
                if (!f) sc = su + sc;
                f = f || fu;
            }
        }
        // exclusive value within the wave
        T ex_s = __shfl_up(sc, 1, 64);
        bool ex_f = __shfl_up((int)f, 1, 64) != 0;
        if (lane == 63) {
            cg_merge_f[wave] = f ? 1.0 : 0.0;
            cg_merge_s[wave] = (double)sc;
        }
        __syncthreads();
        // carry entering this wave: the tile carry, then waves 0 .. wave-1
        T pre = tile_carry;
        for (int w = 0; w < wave; ++w) pre = cg_merge_f[w] != 0.0 ? (T)cg_merge_s[w] : pre + (T)cg_merge_s[w];
        T all = pre;
        for (int w = wave; w < CG_WAVES; ++w) all = cg_merge_f[w] != 0.0 ? (T)cg_merge_s[w] : all + (T)cg_merge_s[w];
        const T incoming = lane == 0 ? pre : (ex_f ? ex_s : pre + ex_s);
        if (first_row >= 0) sink(sl.r0 + first_row, incoming + first_val);
        tile_carry = all;
        __syncthreads();   // the wave sums are read before the next tile writes them
    }
}

// SpMV over the workgroup's rows in whichever layout the slice uses.
template <int U, bool MERGE, typename T, typename F, typename S>
__device__ __forceinline__ void spmv_slice(CInst &p, const Slice &sl, const T *val, const T *sval,
                                           const int *scol, F fetch, S sink) {
    if (MERGE && sl.merge) {
        if constexpr (MERGE) spmv_merge(p, sl, val, fetch, sink);
    } else if (sl.sell) {
        // chunk c on wave c % CG_WAVES, whether it is held in LDS or not: in
        // natural order thread tid computes rows r0 + tid + CG_THREADS * j
        const int lane = threadIdx.x & 63, wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
        for (int c = wave; c < sl.nch; c += CG_WAVES) {
            const int r = 64 * c + lane;
            const int i = sl.perm ? (sl.r0 + r < sl.r1 ? sl.perm[r] : sl.r1) : sl.r0 + r;
            const T acc = c < sl.cc ? sell_chunk<true>(sl, sval, scol, c, lane, fetch)
                                    : sell_chunk<false>(sl, sval, scol, c, lane, fetch);
            if (i < sl.r1) sink(i, acc);
        }
    } else {
        spmv_rows<U>(p.rowptr, p.colind, val, sl.r0, sl.rc, sl.r1, sl.L, sl.kbase, fetch, sink);
    }
}

// FP64 persistent CG with register-resident own rows (see CG_REF_WAVES): r,
// p, q (and D^{-1} for Jacobi) of the thread's rows stay in registers for the
// whole solve; z = D^{-1} r is formed where it is used.  Only p is published
// (the SpMV gathers it) and x is updated in memory (the true residual gathers
// it).  The arithmetic and its order are those of the memory-resident solver
// below, row for row and sum for sum, so both give the same bits.
//
// Every workgroup's slice must be in natural-order sliced ELL with at most
// CG_RV rows per reference thread; when one is not, every workgroup leaves
// after the first barrier with result status CG_STATUS_NOREG and the host
// runs the memory-resident solver instead.
constexpr int CG_STATUS_NOREG = 4;

template <bool JACOBI, class Sync>
__device__ __forceinline__ void cg_f64_reg(CInst *pin, Sync &gs, const int g, const int G) {
    constexpr int M = CG_VT * CG_RV;
    CInst *pp = opaque(pin);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const Slice sl = load_slice(*pp, pp->val, pp->sval64, pp->scol, g, G);
    const int r0 = sl.r0, r1 = sl.r1;
    if (JACOBI) {
        for (int i = r0 + tid; i < r1; i += CG_THREADS) {
            double dg = 0.0;
            for (int k = pp->rowptr[i]; k < pp->rowptr[i + 1]; ++k)
                if (pp->colind[k] == i) dg += pp->val[k];
            pp->dinv[i] = 1.0 / dg;
        }
    }
    {
        const bool fits = sl.sell && !sl.perm && sl.nch <= CG_REF_WAVES * CG_RV;
        if (tid == 0) st_coh(pp->part + (size_t)PART_TRUE * G + g, fits ? 1.0 : 0.0);
        gs.template sync<true>();   // also publishes dinv within the workgroup
        if (grid_total(pp->part, PART_TRUE, G, &cg_bcast) != (double)G) {
            if (g == 0 && tid == 0) {
                pp->result[0] = 0;
                pp->result[1] = CG_STATUS_NOREG;
            }
            return;
        }
    }
    double rv[M], pv[M], qv[M], dv[M];
    static_for<0, M>([&](auto mc) {
        constexpr int m = decltype(mc)::value;
        const int i = reg_row(r0, wave, lane, m);
        rv[m] = pv[m] = qv[m] = 0.0;
        dv[m] = (JACOBI && i < r1) ? pp->dinv[i] : 1.0;
    });
    int k = 0, status = 1, restarts = 0, k_cycle = -1, cap = 0;
    while (cap < pp->ncap && pp->cap_iters[cap] <= 0) ++cap;
    double bnorm = 0.0, rr = 0.0, tt = 0.0;
    for (;;) {
        pp = opaque(pin);
        // phase 0: r = b - A x, p_{-1} = 0, partials b.b, r.z, r.r
        double acc0[CG_VT][3] = {};
        spmv_sell_reg(sl, (const double *)pp->sval64, pp->scol, [&](int c) { return pp->x[c]; },
                      [&](auto mc, int i, double s) { qv[decltype(mc)::value] = s; });
        {
            const int lb = launder_v(lane);
            static_for<0, M>([&](auto mc) {
                constexpr int m = decltype(mc)::value, h = m / CG_RV;
                const int i = reg_row(r0, wave, lb, m);
                if (i < r1) {
                    const double bi = pp->b[i];
                    const double ri = bi - qv[m];
                    const double zi = JACOBI ? dv[m] * ri : ri;
                    rv[m] = ri;
                    pv[m] = 0.0;
                    acc0[h][0] = __builtin_fma(bi, bi, acc0[h][0]);
                    acc0[h][1] = __builtin_fma(ri, zi, acc0[h][1]);
                    acc0[h][2] = __builtin_fma(ri, ri, acc0[h][2]);
                }
            });
        }
        block_sum_ref<3>(acc0);
        if (tid == 0) {
            st_coh(pp->part + (size_t)PART_BB * G + g, acc0[0][0]);
            st_coh(pp->part + (size_t)PART_RZ * G + g, acc0[0][1]);
            st_coh(pp->part + (size_t)PART_RR * G + g, acc0[0][2]);
        }
        gs.template sync<true>();
        bnorm = sqrt(grid_total(pp->part, PART_BB, G, &cg_bcast));
        double rho = grid_total(pp->part, PART_RZ, G, &cg_bcast);
        rr = grid_total(pp->part, PART_RR, G, &cg_bcast);
        if (bnorm == 0.0) {
            for (int i = r0 + tid; i < r1; i += CG_THREADS) st_coh(pp->x + i, 0.0);
            status = 0;
            tt = 0.0;
            break;
        }
        double beta = 0.0;
        while (true) {
            if (sqrt(rr) <= pp->tol * bnorm) break;
            if (k >= pp->maxit) break;
            pp = opaque(pin);
            // phase P: p = z + beta p on own rows, published for the gathers
            double *pn = pp->p;
            {
                const int lb = launder_v(lane);
                static_for<0, M>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
                    const int i = reg_row(r0, wave, lb, m);
                    const double zi = JACOBI ? dv[m] * rv[m] : rv[m];
                    pv[m] = __builtin_fma(beta, pv[m], zi);
                    if (i < r1) st_coh(pn + i, pv[m]);
                });
            }
            gs.template sync<true>();
            // phase 1: q = A p, partial p.q
            double acc1[CG_VT][1] = {};
            spmv_sell_reg(sl, (const double *)pp->sval64, pp->scol, [&](int c) { return pn[c]; },
                          [&](auto mc, int i, double s) {
                              constexpr int m = decltype(mc)::value, h = m / CG_RV;
                              qv[m] = s;
                              acc1[h][0] = __builtin_fma(pv[m], s, acc1[h][0]);
                          });
            block_sum_ref<1>(acc1);
            if (tid == 0) st_coh(pp->part + (size_t)PART_PQ * G + g, acc1[0][0]);
            gs.template sync<true>();
            const double pq = grid_total(pp->part, PART_PQ, G, &cg_bcast);
            if (!(pq > 0.0) || !isfinite(pq)) { status = 2; break; }
            const double alpha = rho / pq;
            pp = opaque(pin);
            // phase 2: x, r updates on own rows, partials r.z, r.r
            double acc2[CG_VT][2] = {};
            const int lb = launder_v(lane);
            static_for<0, M>([&](auto mc) {
                constexpr int m = decltype(mc)::value, h = m / CG_RV;
                const int i = reg_row(r0, wave, lb, m);
                if (i < r1) {
                    st_coh(pp->x + i, __builtin_fma(alpha, pv[m], pp->x[i]));
                    const double ri = __builtin_fma(-alpha, qv[m], rv[m]);
                    rv[m] = ri;
                    const double zi = JACOBI ? dv[m] * ri : ri;
                    acc2[h][0] = __builtin_fma(ri, zi, acc2[h][0]);
                    acc2[h][1] = __builtin_fma(ri, ri, acc2[h][1]);
                }
            });
            block_sum_ref<2>(acc2);
            if (tid == 0) {
                st_coh(pp->part + (size_t)PART_RZ * G + g, acc2[0][0]);
                st_coh(pp->part + (size_t)PART_RR * G + g, acc2[0][1]);
            }
            gs.template sync<true>();
            const double rho_new = grid_total(pp->part, PART_RZ, G, &cg_bcast);
            rr = grid_total(pp->part, PART_RR, G, &cg_bcast);
            ++k;
            if (cap < pp->ncap && k == pp->cap_iters[cap]) {
                static_for<0, M>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
                    const int i = reg_row(r0, wave, lb, m);
                    if (i < r1) {
                        pp->cap_x[(size_t)cap * pp->n + i] = pp->x[i];
                        pp->cap_r[(size_t)cap * pp->n + i] = rv[m];
                    }
                });
                ++cap;
            }
            if (JACOBI && !(rho_new > 0.0) && rr > 0.0) { status = 2; break; }
            beta = rho_new / rho;
            rho = rho_new;
        }
        // true residual ||b - A x|| (x of other workgroups read after the barrier)
        pp = opaque(pin);
        double acc3[CG_VT][1] = {};
        gs.template sync<true>();
        spmv_sell_reg(sl, (const double *)pp->sval64, pp->scol, [&](int c) { return pp->x[c]; },
                      [&](auto mc, int i, double s) {
                          constexpr int h = decltype(mc)::value / CG_RV;
                          const double d = pp->b[i] - s;
                          acc3[h][0] = __builtin_fma(d, d, acc3[h][0]);
                      });
        block_sum_ref<1>(acc3);
        if (tid == 0) st_coh(pp->part + (size_t)PART_TRUE * G + g, acc3[0][0]);
        gs.template sync<true>();
        tt = grid_total(pp->part, PART_TRUE, G, &cg_bcast);
        if (status == 2) break;
        if (sqrt(tt) <= pp->tol * bnorm) { status = 0; break; }
        if (k >= pp->maxit || k == k_cycle) { status = 1; break; }
        k_cycle = k;
        ++restarts;
    }
    if (g == 0 && tid == 0) {
        pp->result[0] = k;
        pp->result[1] = status;
        pp->result[2] = bnorm > 0.0 ? sqrt(rr) / bnorm : 0.0;
        pp->result[3] = bnorm > 0.0 ? sqrt(tt) / bnorm : 0.0;
        pp->result[4] = bnorm;
        pp->result[5] = restarts;
    }
}

// FP64 persistent CG of one problem by a group of G workgroups (this one of
// rank g) synchronised by `gs`.  Per iteration: phase 1 q = A p and p.q,
// phase 2 x, r, z updates and r.z, r.r, each followed by a group barrier and
// a fixed-order all-reduce; before phase 1, phase P updates p in place on
// own rows and a third barrier publishes it.  When the
// recursive residual meets tol the true residual is recomputed; if it fails,
// CG restarts from the current x while iterations remain.
template <bool JACOBI, bool MERGE, class Sync>
__device__ __forceinline__ void cg_f64_body(CInst *pin, Sync &gs, const int g, const int G) {
    // The problem is read from global memory through a pointer laundered at
    // every phase: its fields are reloaded (scalar loads) instead of being
    // kept live in scalar registers across the whole solve.
    CInst *pp = opaque(pin);
    const int tid = threadIdx.x;
    const Slice sl = load_slice<double, MERGE>(*pp, pp->val, pp->sval64, pp->scol, g, G);
    const int r0 = sl.r0, r1 = sl.r1;
    if (JACOBI) {
        for (int i = r0 + tid; i < r1; i += CG_THREADS) {
            double dg = 0.0;
            for (int k = pp->rowptr[i]; k < pp->rowptr[i + 1]; ++k)
                if (pp->colind[k] == i) dg += pp->val[k];
            pp->dinv[i] = 1.0 / dg;
        }
    }
    const double *zsrc = JACOBI ? pp->z : pp->r;
    int k = 0, status = 1, restarts = 0, k_cycle = -1, cap = 0;
    while (cap < pp->ncap && pp->cap_iters[cap] <= 0) ++cap;
    double bnorm = 0.0, rr = 0.0, tt = 0.0;
    for (;;) {
        pp = opaque(pin);
        // phase 0: r = b - A x, z, p_{-1} = 0, partials b.b, r.z, r.r
        double acc0[3] = {0.0, 0.0, 0.0};
        spmv_slice<CG_U, MERGE>(*pp, sl, pp->val, (const double *)pp->sval64, pp->scol, [&](int c) { return pp->x[c]; },
                        [&](int i, double s) { pp->q[i] = s; });
        __syncthreads();
        for (int i = r0 + tid; i < r1; i += CG_THREADS) {
            const double bi = pp->b[i];
            const double ri = bi - pp->q[i];
            const double zi = JACOBI ? pp->dinv[i] * ri : ri;
            if (JACOBI) {
                pp->r[i] = ri;            // read back only by this thread
                st_coh(pp->z + i, zi);    // gathered by other workgroups
            } else {
                st_coh(pp->r + i, ri);
            }
            st_coh(pp->p + i, 0.0);
            acc0[0] = __builtin_fma(bi, bi, acc0[0]);
            acc0[1] = __builtin_fma(ri, zi, acc0[1]);
            acc0[2] = __builtin_fma(ri, ri, acc0[2]);
        }
        block_sum<3>(acc0, cg_red);
        if (tid == 0) {
            st_coh(pp->part + (size_t)PART_BB * G + g, acc0[0]);
            st_coh(pp->part + (size_t)PART_RZ * G + g, acc0[1]);
            st_coh(pp->part + (size_t)PART_RR * G + g, acc0[2]);
        }
        gs.template sync<true>();
        bnorm = sqrt(grid_total(pp->part, PART_BB, G, &cg_bcast));
        double rho = grid_total(pp->part, PART_RZ, G, &cg_bcast);
        rr = grid_total(pp->part, PART_RR, G, &cg_bcast);
        if (bnorm == 0.0) {
            for (int i = r0 + tid; i < r1; i += CG_THREADS) st_coh(pp->x + i, 0.0);
            status = 0;
            tt = 0.0;
            break;
        }
        double beta = 0.0;
        while (true) {
            if (sqrt(rr) <= pp->tol * bnorm) break;
            if (k >= pp->maxit) break;
            pp = opaque(pin);
            double acc1[1] = {0.0};
            double *pn = pp->p;
            for (int i = r0 + tid; i < r1; i += CG_THREADS) st_coh(pn + i, __builtin_fma(beta, pn[i], zsrc[i]));
            gs.template sync<true>();
            spmv_slice<CG_U, MERGE>(*pp, sl, pp->val, (const double *)pp->sval64, pp->scol, [&](int c) { return pn[c]; },
                            [&](int i, double s) {
                                pp->q[i] = s;
                                acc1[0] = __builtin_fma(pn[i], s, acc1[0]);
                            });
            block_sum<1>(acc1, cg_red);
            if (tid == 0) st_coh(pp->part + (size_t)PART_PQ * G + g, acc1[0]);
            gs.template sync<true>();
            const double pq = grid_total(pp->part, PART_PQ, G, &cg_bcast);
            if (!(pq > 0.0) || !isfinite(pq)) { status = 2; break; }
            const double alpha = rho / pq;
            pp = opaque(pin);
            // phase 2: x, r, z updates on own rows
            double acc2[2] = {0.0, 0.0};
            for (int i = r0 + tid; i < r1; i += CG_THREADS) {
                const double pi = pn[i], qi = pp->q[i], xi = pp->x[i], ro = pp->r[i];
                st_coh(pp->x + i, __builtin_fma(alpha, pi, xi));   // read by others at exit
                const double ri = __builtin_fma(-alpha, qi, ro);
                double zi = ri;
                if (JACOBI) {
                    pp->r[i] = ri;
                    zi = pp->dinv[i] * ri;
                    st_coh(pp->z + i, zi);
                } else {
                    st_coh(pp->r + i, ri);
                }
                acc2[0] = __builtin_fma(ri, zi, acc2[0]);
                acc2[1] = __builtin_fma(ri, ri, acc2[1]);
            }
            block_sum<2>(acc2, cg_red);
            if (tid == 0) {
                st_coh(pp->part + (size_t)PART_RZ * G + g, acc2[0]);
                st_coh(pp->part + (size_t)PART_RR * G + g, acc2[1]);
            }
            gs.template sync<true>();
            const double rho_new = grid_total(pp->part, PART_RZ, G, &cg_bcast);
            rr = grid_total(pp->part, PART_RR, G, &cg_bcast);
            ++k;
            if (cap < pp->ncap && k == pp->cap_iters[cap]) {
                // snapshot of the iterate and its residual (own rows, same
                // thread-to-row mapping as phase 2)
                for (int i = r0 + tid; i < r1; i += CG_THREADS) {
                    pp->cap_x[(size_t)cap * pp->n + i] = pp->x[i];
                    pp->cap_r[(size_t)cap * pp->n + i] = pp->r[i];
                }
                ++cap;
            }
            if (JACOBI && !(rho_new > 0.0) && rr > 0.0) { status = 2; break; }
            beta = rho_new / rho;
            rho = rho_new;
        }
        // true residual ||b - A x|| (x of other workgroups read after the barrier)
        pp = opaque(pin);
        double acc3[1] = {0.0};
        gs.template sync<true>();
        spmv_slice<CG_U, MERGE>(*pp, sl, pp->val, (const double *)pp->sval64, pp->scol, [&](int c) { return pp->x[c]; },
                        [&](int i, double s) {
                            const double d = pp->b[i] - s;
                            acc3[0] = __builtin_fma(d, d, acc3[0]);
                        });
        block_sum<1>(acc3, cg_red);
        if (tid == 0) st_coh(pp->part + (size_t)PART_TRUE * G + g, acc3[0]);
        gs.template sync<true>();
        tt = grid_total(pp->part, PART_TRUE, G, &cg_bcast);
        if (status == 2) break;
        if (sqrt(tt) <= pp->tol * bnorm) { status = 0; break; }
        // restart from x (recursive residual converged but the true one did
        // not) unless the iteration budget is spent or the last cycle made no
        // iteration (the two residuals differ only in rounding order there)
        if (k >= pp->maxit || k == k_cycle) { status = 1; break; }
        k_cycle = k;
        ++restarts;
    }
    if (g == 0 && tid == 0) {
        pp->result[0] = k;
        pp->result[1] = status;
        pp->result[2] = bnorm > 0.0 ? sqrt(rr) / bnorm : 0.0;
        pp->result[3] = bnorm > 0.0 ? sqrt(tt) / bnorm : 0.0;
        pp->result[4] = bnorm;
        pp->result[5] = restarts;
    }
}

// Mixed precision: one FP32 CG recurrence whose recursive residual is
// replaced, from time to time, by the true residual of an FP64 iterate
// (residual replacement, "reliable updates"), the search direction being kept
// across each replacement so that the Krylov space built so far survives.
//   replacement (FP64): x += d / s on own rows; r = b - A x with the FP64
//     matrix; stop when ||r|| <= tol ||b||; new exact scale s' = 2^-floor(
//     log2 ||r||); r32 = float(s' r), z32, d = 0, p32 *= s'/s (exact), and
//     beta = (r32, z32) / (rho (s'/s)^2) (the first replacement: p = z).
//   iteration (FP32 vectors, SpMV and AXPYs; FP64 dots, alpha, beta), until
//     ||r32|| <= update_tol * (its largest value since the replacement), or
//     ||r32|| / s <= tol ||b||, or the budget is spent, or a breakdown.
//   stagnation: PERKS_MIXED_STALL replacements in a row without a new
//     smallest true residual end the solve (FP32 cannot resolve the system).
// Barriers: three per iteration (as the FP64 solver) and three per
// replacement.  The FP32 copy of each workgroup's slice of A is made by the
// workgroup itself (global copy + LDS cache of its first CG_LDS_NNZ32
// entries): 8 instead of 12 bytes per nonzero in the FP32 iterations, and
// 1.5x the nonzeros held on chip.
template <bool JACOBI, bool MERGE, class Sync>
__device__ __forceinline__ void cg_mixed_body(CInst &p, Sync &gs, const int g, const int G) {
    const int tid = threadIdx.x;
    {
        // FP32 copy of this workgroup's slice (only this workgroup reads it)
        const int s0 = p.rowptr[merge_split(p.rowptr, p.n, p.nnz, g, G)];
        const int s1 = p.rowptr[merge_split(p.rowptr, p.n, p.nnz, g + 1, G)];
        for (int k = s0 + tid; k < s1; k += CG_THREADS) p.val32[k] = (float)p.val[k];
    }
    // its barriers publish val32
    const Slice sl = load_slice<float, MERGE>(p, (const float *)p.val32, p.sval32, p.scol, g, G, p.sval64);
    const int r0 = sl.r0, r1 = sl.r1, kbase = sl.kbase, L = sl.L;
    Slice s64 = sl;
    s64.cc = 0;   // the FP64 sliced-ELL values are read from global memory only
    double accb[1] = {0.0};
    for (int i = r0 + tid; i < r1; i += CG_THREADS) {
        if (JACOBI) {
            double dg = 0.0;
            for (int k = p.rowptr[i]; k < p.rowptr[i + 1]; ++k)
                if (p.colind[k] == i) dg += p.val[k];
            p.dinv32[i] = (float)(1.0 / dg);
        }
        const double bi = p.b[i];
        accb[0] = __builtin_fma(bi, bi, accb[0]);
        p.d32[i] = 0.0f;
        p.p32[i] = 0.0f;
    }
    block_sum<1>(accb, cg_red);
    if (tid == 0) st_coh(p.part + (size_t)PART_BB * G + g, accb[0]);

    const float *zsrc = JACOBI ? p.z32 : p.r32;
    double bnorm = -1.0, rn = 0.0, best = INFINITY, sc = 1.0, rho = 0.0;
    int k = 0, outer = 0, status = 1, stall = 0;
    bool broke = false;
    for (;;) {
        // replacement: fold the FP32 correction into x (own rows; every
        // workgroup reads x in the residual below)
        for (int i = r0 + tid; i < r1; i += CG_THREADS) st_coh(p.x + i, p.x[i] + (double)p.d32[i] / sc);
        gs.template sync<true>();   // x (and, the first time, the b.b partials) complete
        if (bnorm < 0.0) bnorm = sqrt(grid_total(p.part, PART_BB, G, &cg_bcast));
        if (bnorm == 0.0) {
            for (int i = r0 + tid; i < r1; i += CG_THREADS) st_coh(p.x + i, 0.0);
            status = 0;
            rn = 0.0;
            break;
        }
        // true residual in FP64 (A from global memory in FP64: its sliced-ELL
        // copy when the slice has that layout, else CSR)
        double accr[1] = {0.0};
        {
            auto fx = [&](int c) { return p.x[c]; };
            auto sink = [&](int i, double sv) {
                const double ri = p.b[i] - sv;
                p.r64[i] = ri;
                accr[0] = __builtin_fma(ri, ri, accr[0]);
            };
            if (sl.sell) spmv_slice<CG_U, false>(p, s64, p.val, (const double *)p.sval64, p.scol, fx, sink);
            else spmv_range<CG_U, false>(p.rowptr, p.colind, p.val, r0, r1, L, kbase, fx, sink);
        }
        block_sum<1>(accr, cg_red);
        if (tid == 0) st_coh(p.part + (size_t)PART_TRUE * G + g, accr[0]);
        gs.template sync<true>();
        rn = sqrt(grid_total(p.part, PART_TRUE, G, &cg_bcast));
        if (rn <= p.tol * bnorm) { status = 0; break; }
        if (broke) { status = 2; break; }
        if (rn < best) {
            best = rn;
            stall = 0;
        } else if (++stall >= PERKS_MIXED_STALL) {
            break;
        }
        if (k >= p.maxit || outer >= p.max_outer) break;
        // restart the recurrence's residual from r, keep its direction
        int ex;
        (void)frexp(rn, &ex);
        const double sc_new = ldexp(1.0, 1 - ex);   // 2^-floor(log2 rn)
        const double ratio = outer == 0 ? 1.0 : sc_new / sc;   // first: p is 0
        const float ratio_f = (float)ratio;
        double acc0[2] = {0.0, 0.0};
        for (int i = r0 + tid; i < r1; i += CG_THREADS) {
            const float ri = (float)(p.r64[i] * sc_new);
            const float zi = JACOBI ? p.dinv32[i] * ri : ri;
            if (JACOBI) {
                p.r32[i] = ri;
                st_coh(p.z32 + i, zi);
            } else {
                st_coh(p.r32 + i, ri);
            }
            p.p32[i] = p.p32[i] * ratio_f;   // own rows, read back by this thread in phase P
            p.d32[i] = 0.0f;
            acc0[0] = __builtin_fma((double)ri, (double)zi, acc0[0]);
            acc0[1] = __builtin_fma((double)ri, (double)ri, acc0[1]);
        }
        block_sum<2>(acc0, cg_red);
        if (tid == 0) {
            st_coh(p.part + (size_t)PART_RZ * G + g, acc0[0]);
            st_coh(p.part + (size_t)PART_RR * G + g, acc0[1]);
        }
        gs.template sync<true>();
        const double rho_r = grid_total(p.part, PART_RZ, G, &cg_bcast);
        double beta = outer == 0 ? 0.0 : rho_r / (rho * ratio * ratio);
        rho = rho_r;
        sc = sc_new;
        double rmax = sqrt(grid_total(p.part, PART_RR, G, &cg_bcast));
        // FP32 iterations until the next replacement
        for (;;) {
            const float bf = (float)beta;
            double acc1[1] = {0.0};
            float *pn = p.p32;
            for (int i = r0 + tid; i < r1; i += CG_THREADS) st_coh(pn + i, __builtin_fmaf(bf, pn[i], zsrc[i]));
            gs.template sync<true>();
            spmv_slice<CG_U, MERGE>(p, sl, (const float *)p.val32, (const float *)p.sval32, p.scol,
                            [&](int c) { return pn[c]; },
                            [&](int i, float sv) {
                                p.q32[i] = sv;
                                acc1[0] = __builtin_fma((double)pn[i], (double)sv, acc1[0]);
                            });
            block_sum<1>(acc1, cg_red);
            if (tid == 0) st_coh(p.part + (size_t)PART_PQ * G + g, acc1[0]);
            gs.template sync<true>();
            const double pq = grid_total(p.part, PART_PQ, G, &cg_bcast);
            if (!(pq > 0.0) || !isfinite(pq)) { broke = true; break; }
            const float af = (float)(rho / pq);
            double acc2[2] = {0.0, 0.0};
            for (int i = r0 + tid; i < r1; i += CG_THREADS) {
                const float pi = pn[i];
                p.d32[i] = __builtin_fmaf(af, pi, p.d32[i]);
                const float ri = __builtin_fmaf(-af, p.q32[i], p.r32[i]);
                float zi = ri;
                if (JACOBI) {
                    p.r32[i] = ri;
                    zi = p.dinv32[i] * ri;
                    st_coh(p.z32 + i, zi);
                } else {
                    st_coh(p.r32 + i, ri);
                }
                acc2[0] = __builtin_fma((double)ri, (double)zi, acc2[0]);
                acc2[1] = __builtin_fma((double)ri, (double)ri, acc2[1]);
            }
            block_sum<2>(acc2, cg_red);
            if (tid == 0) {
                st_coh(p.part + (size_t)PART_RZ * G + g, acc2[0]);
                st_coh(p.part + (size_t)PART_RR * G + g, acc2[1]);
            }
            gs.template sync<true>();
            const double rho_new = grid_total(p.part, PART_RZ, G, &cg_bcast);
            const double rnorm = sqrt(grid_total(p.part, PART_RR, G, &cg_bcast));
            ++k;
            if (JACOBI && !(rho_new > 0.0) && rnorm > 0.0) { broke = true; break; }
            rmax = fmax(rmax, rnorm);
            if (rnorm <= p.update_tol * rmax || rnorm <= p.tol * bnorm * sc || k >= p.maxit) break;
            beta = rho_new / rho;
            rho = rho_new;
        }
        ++outer;
    }
    if (g == 0 && tid == 0) {
        p.result[0] = k;
        p.result[1] = status;
        p.result[2] = bnorm > 0.0 ? rn / bnorm : 0.0;
        p.result[3] = bnorm > 0.0 ? rn / bnorm : 0.0;
        p.result[4] = bnorm;
        p.result[5] = outer;
    }
}

// Mixed-precision persistent CG with register-resident own rows: the FP32
// r, p, q, d (and D^{-1}) of the thread's rows stay in registers for the whole
// solve (see CG_REF_WAVES for the row mapping), so an FP32 iteration moves
// A's values beyond the LDS copy, p once published and once gathered, and
// nothing else; x and the FP64 residual are touched only at replacements.
// The arithmetic and its order are those of cg_mixed_body, row for row and
// sum for sum, so both give the same bits.  The same eligibility rule as
// cg_f64_reg (CG_STATUS_NOREG when a slice does not allow it).
template <bool JACOBI, class Sync>
__device__ __forceinline__ void cg_mixed_reg(CInst *pin, Sync &gs, const int g, const int G) {
    constexpr int M = CG_VT * CG_RV;
    CInst *pp = opaque(pin);
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    {
        const int s0 = pp->rowptr[merge_split(pp->rowptr, pp->n, pp->nnz, g, G)];
        const int s1 = pp->rowptr[merge_split(pp->rowptr, pp->n, pp->nnz, g + 1, G)];
        for (int k = s0 + tid; k < s1; k += CG_THREADS) pp->val32[k] = (float)pp->val[k];
    }
    const Slice sl = load_slice<float>(*pp, (const float *)pp->val32, pp->sval32, pp->scol, g, G, pp->sval64);
    const int r0 = sl.r0, r1 = sl.r1;
    Slice s64 = sl;
    s64.cc = 0;
    float rv[M], pv[M], qv[M], dv[M], wv[M];
    double accb[CG_VT][1] = {};
    {
        const int lb = launder_v(lane);
        static_for<0, M>([&](auto mc) {
            constexpr int m = decltype(mc)::value, h = m / CG_RV;
            const int i = reg_row(r0, wave, lb, m);
            rv[m] = pv[m] = qv[m] = dv[m] = 0.0f;
            wv[m] = 1.0f;
            if (i < r1) {
                if (JACOBI) {
                    double dg = 0.0;
                    for (int k = pp->rowptr[i]; k < pp->rowptr[i + 1]; ++k)
                        if (pp->colind[k] == i) dg += pp->val[k];
                    wv[m] = (float)(1.0 / dg);
                }
                const double bi = pp->b[i];
                accb[h][0] = __builtin_fma(bi, bi, accb[h][0]);
            }
        });
    }
    block_sum_ref<1>(accb);
    {
        const bool fits = sl.sell && !sl.perm && sl.nch <= CG_REF_WAVES * CG_RV;
        if (tid == 0) {
            st_coh(pp->part + (size_t)PART_TRUE * G + g, fits ? 1.0 : 0.0);
            st_coh(pp->part + (size_t)PART_BB * G + g, accb[0][0]);
        }
        gs.template sync<true>();
        if (grid_total(pp->part, PART_TRUE, G, &cg_bcast) != (double)G) {
            if (g == 0 && tid == 0) {
                pp->result[0] = 0;
                pp->result[1] = CG_STATUS_NOREG;
            }
            return;
        }
    }
    const double bnorm = sqrt(grid_total(pp->part, PART_BB, G, &cg_bcast));
    double rn = 0.0, best = INFINITY, sc = 1.0, rho = 0.0;
    int k = 0, outer = 0, status = 1, stall = 0;
    bool broke = false;
    for (;;) {
        pp = opaque(pin);
        // replacement: fold the FP32 correction into x (own rows)
        {
            const int lb = launder_v(lane);
            static_for<0, M>([&](auto mc) {
                constexpr int m = decltype(mc)::value;
                const int i = reg_row(r0, wave, lb, m);
                if (i < r1) st_coh(pp->x + i, pp->x[i] + (double)dv[m] / sc);
            });
        }
        gs.template sync<true>();
        if (bnorm == 0.0) {
            for (int i = r0 + tid; i < r1; i += CG_THREADS) st_coh(pp->x + i, 0.0);
            status = 0;
            rn = 0.0;
            break;
        }
        // true residual in FP64 (sliced-ELL FP64 values from global memory);
        // r64 of own rows kept in memory until the new scale is known
        double accr[CG_VT][1] = {};
        spmv_sell_reg(s64, (const double *)pp->sval64, pp->scol, [&](int c) { return pp->x[c]; },
                      [&](auto mc, int i, double sv) {
                          constexpr int h = decltype(mc)::value / CG_RV;
                          const double ri = pp->b[i] - sv;
                          pp->r64[i] = ri;
                          accr[h][0] = __builtin_fma(ri, ri, accr[h][0]);
                      });
        block_sum_ref<1>(accr);
        if (tid == 0) st_coh(pp->part + (size_t)PART_TRUE * G + g, accr[0][0]);
        gs.template sync<true>();
        rn = sqrt(grid_total(pp->part, PART_TRUE, G, &cg_bcast));
        if (rn <= pp->tol * bnorm) { status = 0; break; }
        if (broke) { status = 2; break; }
        if (rn < best) {
            best = rn;
            stall = 0;
        } else if (++stall >= PERKS_MIXED_STALL) {
            break;
        }
        if (k >= pp->maxit || outer >= pp->max_outer) break;
        int ex;
        (void)frexp(rn, &ex);
        const double sc_new = ldexp(1.0, 1 - ex);   // 2^-floor(log2 rn)
        const double ratio = outer == 0 ? 1.0 : sc_new / sc;   // first: p is 0
        const float ratio_f = (float)ratio;
        double acc0[CG_VT][2] = {};
        {
            const int lb = launder_v(lane);
            static_for<0, M>([&](auto mc) {
                constexpr int m = decltype(mc)::value, h = m / CG_RV;
                const int i = reg_row(r0, wave, lb, m);
                if (i < r1) {
                    const float ri = (float)(pp->r64[i] * sc_new);
                    const float zi = JACOBI ? wv[m] * ri : ri;
                    rv[m] = ri;
                    pv[m] = pv[m] * ratio_f;
                    dv[m] = 0.0f;
                    acc0[h][0] = __builtin_fma((double)ri, (double)zi, acc0[h][0]);
                    acc0[h][1] = __builtin_fma((double)ri, (double)ri, acc0[h][1]);
                }
            });
        }
        block_sum_ref<2>(acc0);
        if (tid == 0) {
            st_coh(pp->part + (size_t)PART_RZ * G + g, acc0[0][0]);
            st_coh(pp->part + (size_t)PART_RR * G + g, acc0[0][1]);
        }
        gs.template sync<true>();
        const double rho_r = grid_total(pp->part, PART_RZ, G, &cg_bcast);
        double beta = outer == 0 ? 0.0 : rho_r / (rho * ratio * ratio);
        rho = rho_r;
        sc = sc_new;
        double rmax = sqrt(grid_total(pp->part, PART_RR, G, &cg_bcast));
        for (;;) {
            pp = opaque(pin);
            // phase P: p = z + beta p on own rows, published for the gathers
            const float bf = (float)beta;
            float *pn = pp->p32;
            {
                const int lb = launder_v(lane);
                static_for<0, M>([&](auto mc) {
                    constexpr int m = decltype(mc)::value;
                    const int i = reg_row(r0, wave, lb, m);
                    const float zi = JACOBI ? wv[m] * rv[m] : rv[m];
                    pv[m] = __builtin_fmaf(bf, pv[m], zi);
                    if (i < r1) st_coh(pn + i, pv[m]);
                });
            }
            gs.template sync<true>();
            // phase 1: q = A p (FP32), partial p.q in FP64
            double acc1[CG_VT][1] = {};
            spmv_sell_reg(sl, (const float *)pp->sval32, pp->scol, [&](int c) { return pn[c]; },
                          [&](auto mc, int i, float sv) {
                              constexpr int m = decltype(mc)::value, h = m / CG_RV;
                              qv[m] = sv;
                              acc1[h][0] = __builtin_fma((double)pv[m], (double)sv, acc1[h][0]);
                          });
            block_sum_ref<1>(acc1);
            if (tid == 0) st_coh(pp->part + (size_t)PART_PQ * G + g, acc1[0][0]);
            gs.template sync<true>();
            const double pq = grid_total(pp->part, PART_PQ, G, &cg_bcast);
            if (!(pq > 0.0) || !isfinite(pq)) { broke = true; break; }
            const float af = (float)(rho / pq);
            // phase 2: d, r updates on own rows, partials r.z, r.r in FP64
            double acc2[CG_VT][2] = {};
            {
                const int lb = launder_v(lane);
                static_for<0, M>([&](auto mc) {
                    constexpr int m = decltype(mc)::value, h = m / CG_RV;
                    const int i = reg_row(r0, wave, lb, m);
                    if (i < r1) {
                        dv[m] = __builtin_fmaf(af, pv[m], dv[m]);
                        const float ri = __builtin_fmaf(-af, qv[m], rv[m]);
                        rv[m] = ri;
                        const float zi = JACOBI ? wv[m] * ri : ri;
                        acc2[h][0] = __builtin_fma((double)ri, (double)zi, acc2[h][0]);
                        acc2[h][1] = __builtin_fma((double)ri, (double)ri, acc2[h][1]);
                    }
                });
            }
            block_sum_ref<2>(acc2);
            if (tid == 0) {
                st_coh(pp->part + (size_t)PART_RZ * G + g, acc2[0][0]);
                st_coh(pp->part + (size_t)PART_RR * G + g, acc2[0][1]);
            }
            gs.template sync<true>();
            const double rho_new = grid_total(pp->part, PART_RZ, G, &cg_bcast);
            const double rnorm = sqrt(grid_total(pp->part, PART_RR, G, &cg_bcast));
            ++k;
            if (JACOBI && !(rho_new > 0.0) && rnorm > 0.0) { broke = true; break; }
            rmax = fmax(rmax, rnorm);
            if (rnorm <= pp->update_tol * rmax || rnorm <= pp->tol * bnorm * sc || k >= pp->maxit) break;
            beta = rho_new / rho;
            rho = rho_new;
        }
        ++outer;
    }
    if (g == 0 && tid == 0) {
        pp->result[0] = k;
        pp->result[1] = status;
        pp->result[2] = bnorm > 0.0 ? rn / bnorm : 0.0;
        pp->result[3] = bnorm > 0.0 ? rn / bnorm : 0.0;
        pp->result[4] = bnorm;
        pp->result[5] = outer;
    }
}

// One problem on the whole grid.
template <bool JACOBI, bool MIXED, bool MERGE>
__global__ __launch_bounds__(CG_THREADS) void cg_persistent(const CgInst *pin, unsigned *ws) {
    BarrierClock clk;
    clk.start();
    GroupSync gs;
    gs.init_grid(ws, &clk);
    CInst *in = (CInst *)pin;
    if (MIXED) cg_mixed_body<JACOBI, MERGE>(*in, gs, blockIdx.x, gridDim.x);
    else cg_f64_body<JACOBI, MERGE>(in, gs, blockIdx.x, gridDim.x);
    if (blockIdx.x == 0 && threadIdx.x == 0) st_coh(ws + SYNC_EPOCH, gs.epoch);
    clk.publish(ws);
}

// One problem on the whole grid, own rows in registers (FP64 or mixed
// precision; status CG_STATUS_NOREG when a slice does not allow it).
// Instantiated by cg_reg.hip only.
template <bool JACOBI, bool MIXED>
__global__ __launch_bounds__(CG_THREADS) void cg_persistent_reg(const CgInst *pin, unsigned *ws) {
    BarrierClock clk;
    clk.start();
    GroupSync gs;
    gs.init_grid(ws, &clk);
    if (MIXED) cg_mixed_reg<JACOBI>((CInst *)pin, gs, blockIdx.x, gridDim.x);
    else cg_f64_reg<JACOBI>((CInst *)pin, gs, blockIdx.x, gridDim.x);
    if (blockIdx.x == 0 && threadIdx.x == 0) st_coh(ws + SYNC_EPOCH, gs.epoch);
    clk.publish(ws);
}

// Many problems in one launch.  Workgroup g runs the tasks
// tasks[task_ptr[g] .. task_ptr[g+1]) in order; a task is (problem, rank,
// group size, group id).  A problem given to several workgroups is the first
// task of each of them (a contiguous range of workgroups, synchronised by the
// group's own barrier); the other problems are solved by one workgroup each,
// one after another.  Every workgroup takes its tasks in the same phase
// order, so no wait can be circular.  A final barrier of the whole grid
// precedes the hand-over of the epoch to the next launch.
struct CgTask {
    int inst, rank, size, group;
};

struct CgBatch {
    const CgInst *inst;
    const CgTask *tasks;
    const int *task_ptr;
    unsigned *ws;
    unsigned epoch_span;   // > barriers any group takes: group j uses epochs start + j*span + 1 ..
    int ngroups;           // groups of two or more workgroups (ids 0 .. ngroups-1)
};

template <bool JACOBI, bool MIXED>
__global__ __launch_bounds__(CG_THREADS) void cg_batched(CgBatch bp) {
    const int g = blockIdx.x;
    BarrierClock clk;
    clk.start();
    const unsigned e0 = ld_coh(bp.ws + SYNC_EPOCH);
    for (int t = bp.task_ptr[g]; t < bp.task_ptr[g + 1]; ++t) {
        const CgTask task = bp.tasks[t];
        GroupSync gs;
        // disjoint epoch ranges per group: a workgroup's flag left by an
        // earlier group can never match a later group's epochs
        gs.init(bp.ws, g - task.rank, task.group, task.rank, task.size, e0 + (unsigned)task.group * bp.epoch_span,
                &clk);
        CInst *in = (CInst *)(bp.inst + task.inst);
        if (MIXED) cg_mixed_body<JACOBI, false>(*in, gs, task.rank, task.size);
        else cg_f64_body<JACOBI, false>(in, gs, task.rank, task.size);
    }
    GroupSync all;
    all.init(bp.ws, 0, 0, g, gridDim.x, e0 + (unsigned)bp.ngroups * bp.epoch_span, &clk);
    all.gen = bp.ws + SYNC_GEN;
    all.sync();
    if (g == 0 && threadIdx.x == 0) st_coh(bp.ws + SYNC_EPOCH, all.epoch);
    clk.publish(bp.ws);
}

}  // namespace
}  // namespace perks
