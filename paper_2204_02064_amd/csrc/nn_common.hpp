// Network constants, bfloat16 conversions and weight packing shared by the
// network kernels and the flexible-CG kernel that applies the network.
#pragma once

#include "common.hpp"

namespace perks {
namespace {

constexpr int NC = 16;                        // channels of every stored activation
constexpr int NL = PERKS_NN_LAYERS;           // 6
constexpr int LAYER_PARAMS = NC * NC * 9 + NC;
constexpr int IN_CH[NL] = {2, 16, 16, 16, 16, 16};
constexpr int OUT_CH[NL] = {16, 16, 16, 16, 16, 1};

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// float -> bfloat16 bits, round to nearest, ties to even (finite inputs).
__device__ __forceinline__ unsigned short to_bf16(float f) {
    unsigned u = __float_as_uint(f);
    u += 0x7FFFu + ((u >> 16) & 1u);
    return (unsigned short)(u >> 16);
}
__device__ __forceinline__ float from_bf16(unsigned short h) { return __uint_as_float((unsigned)h << 16); }

// ---------------------------------------------------------------------------
// Weight packing.  params (FP32, padded): layer l at l * LAYER_PARAMS:
// W[o][i][ty][tx] (16 x 16 x 3 x 3) then b[16].  Fragments: for layer l,
// pass q (0..4), lane: 8 bf16 = A[m = lane%16][k = 8(lane/16) + j], with
// k -> (tap = 2q + k/16, channel = k%16).  Forward: A[o][tap, i] = W[o][i][tap].
// Backward (input gradient): A[i][tap, o] = W[o][i][8 - tap].
__global__ __launch_bounds__(256) void nn_pack(const float *params, unsigned short *wf, unsigned short *wb,
                                               float *bias) {
    const int idx = blockIdx.x * 256 + threadIdx.x;   // (layer, q, lane, j)
    if (idx >= NL * 5 * 64 * 8) return;
    const int j = idx & 7, lane = (idx >> 3) & 63, q = (idx >> 9) % 5, l = idx / (5 * 512);
    const int m = lane & 15, k = 8 * (lane >> 4) + j;
    const int tap = 2 * q + (k >> 4), c = k & 15;
    const float *W = params + (size_t)l * LAYER_PARAMS;
    float f = 0.f, b = 0.f;
    if (tap < 9) {
        f = W[(m * NC + c) * 9 + tap];           // o = m, i = c
        b = W[(c * NC + m) * 9 + (8 - tap)];     // o = c, i = m, flipped tap
    }
    wf[idx] = to_bf16(f);
    wb[idx] = to_bf16(b);
    if (q == 0 && j == 0 && lane < 16) bias[l * NC + lane] = W[NC * NC * 9 + lane];
}

}  // namespace
}  // namespace perks
