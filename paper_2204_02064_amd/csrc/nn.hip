// Learned preconditioner: a six-layer 3x3 convolutional network in BF16 on
// the matrix cores (FP32 accumulate), its training (backward pass, MSE loss,
// Adam) and its application inside flexible CG.  The paper has no learned
// component; this is the extension's hot path.
//
// Network (weights W[o][i][1+dy][1+dx] multiply input channel i at
// (y+dy, x+dx) for output channel o at (y, x); zero 'same' padding; bias;
// ReLU after every layer but the last):
//     [r / rms(r), log k] (2) -> 16 -> 16 -> 16 -> 16 -> 16 -> 1
// Every layer runs as a 16 -> 16 channel layer (unused channels have zero
// weights), so one kernel serves all six.  Activations are stored
// pixel-major with the 16 channels of a pixel contiguous (32 bytes in BF16).
//
// Matrix-core mapping (v_mfma_f32_16x16x32_bf16, D = A B + C, 16 x 16 x 32):
// M = 16 output channels, N = 16 consecutive pixels of a row, K = 32 = two
// taps x 16 input channels; the nine taps take five instructions (the tenth
// tap has zero weights).  Lane l holds A[m = l%16][k = 8(l/16) .. +7] (the
// weights, kept in registers), B[k = 8(l/16) .. +7][n = l%16] (eight
// channels of one input pixel: one 16-byte load) and D[m = 4(l/16) .. +3]
// [n = l%16] (four output channels of one pixel: one 8-byte store).
//
// The input gradient of a layer is the same convolution with the weights
// transposed (o <-> i) and flipped (dy, dx -> -dy, -dx); the weight gradient
// is a per-pixel outer product summed over the image (FP32 vector units,
// partial sums per workgroup, then a fixed-order reduction).
#include <algorithm>
#include <cmath>
#include <vector>

#include "common.hpp"
#include "nn_common.hpp"

namespace perks {
namespace {

// ---------------------------------------------------------------------------
// One 3x3 layer on the matrix cores.  Each wave computes SEG segments of 16
// pixels along x of one row; a workgroup holds 4 waves (4 rows).
//   in      [B][H][W][16] bf16
//   frag    packed A fragments of this layer (5 x 64 x 8 bf16)
//   bias    16 floats or NULL
//   mode    0: out bf16 = relu(conv + bias)
//           1: out f32 = conv + bias, channel 0 only ([B][H][W] floats)
//           2: out bf16 = conv * (mask > 0)   (input gradient through a ReLU)
//           3: out bf16 = conv                (input gradient, no ReLU before)
constexpr int SEG = 4;

__global__ __launch_bounds__(256) void nn_conv(const unsigned short *in, const unsigned short *frag,
                                               const float *bias, const unsigned short *mask, void *out, int B,
                                               int H, int W, int mode) {
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    const int segs = (W + 15) / 16;
    const int xblocks = (segs + SEG - 1) / SEG;
    const int rows = B * H;
    const int row = (blockIdx.x / xblocks) * 4 + wave;
    if (row >= rows) return;
    const int img = row / H, y = row % H;
    const int seg0 = (blockIdx.x % xblocks) * SEG;
    bf16x8 a[5];
    const uint4 *fr = reinterpret_cast<const uint4 *>(frag);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        const uint4 v = fr[q * 64 + lane];
        a[q] = *reinterpret_cast<const bf16x8 *>(&v);
    }
    const int n = lane & 15, g = lane >> 4;
    const int cofs = 8 * (g & 1);   // input channels of this lane's B fragment
    float bz[4] = {0.f, 0.f, 0.f, 0.f};
    if (bias) {
#pragma unroll
        for (int j = 0; j < 4; ++j) bz[j] = bias[4 * g + j];
    }
    const size_t img_base = (size_t)img * H * W;
    for (int s = seg0; s < min(seg0 + SEG, segs); ++s) {
        const int x = s * 16 + n;
        f32x4 acc = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 5; ++q) {
            const int tap = 2 * q + (g >> 1);
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (tap < 9) {
                const int yy = y + tap / 3 - 1, xx = x + tap % 3 - 1;
                if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                    v = *reinterpret_cast<const uint4 *>(in + ((img_base + (size_t)yy * W + xx) * NC + cofs));
            }
            acc = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[q], *reinterpret_cast<const bf16x8 *>(&v), acc, 0, 0, 0);
        }
        if (x >= W) continue;
        const size_t pix = img_base + (size_t)y * W + x;
        if (mode == 1) {
            if (g == 0) reinterpret_cast<float *>(out)[pix] = acc[0] + bz[0];
            continue;
        }
        float o[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) o[j] = acc[j] + bz[j];
        if (mode == 0) {
#pragma unroll
            for (int j = 0; j < 4; ++j) o[j] = fmaxf(o[j], 0.f);
        } else if (mode == 2) {
            const uint2 mk = *reinterpret_cast<const uint2 *>(mask + pix * NC + 4 * g);
            const unsigned short mh[4] = {(unsigned short)(mk.x & 0xFFFF), (unsigned short)(mk.x >> 16),
                                          (unsigned short)(mk.y & 0xFFFF), (unsigned short)(mk.y >> 16)};
#pragma unroll
            for (int j = 0; j < 4; ++j) o[j] = from_bf16(mh[j]) > 0.f ? o[j] : 0.f;
        }
        uint2 st;
        st.x = (unsigned)to_bf16(o[0]) | ((unsigned)to_bf16(o[1]) << 16);
        st.y = (unsigned)to_bf16(o[2]) | ((unsigned)to_bf16(o[3]) << 16);
        *reinterpret_cast<uint2 *>(reinterpret_cast<unsigned short *>(out) + pix * NC + 4 * g) = st;
    }
}

// Network input: channel 0 = bf16(r / rms), channel 1 = bf16(log k), rest 0.
//   x  [B][H][W][2] floats (already scaled), or from FCG (r, logk, 1/rms).
__global__ __launch_bounds__(256) void nn_pack_input(const float *x, int P, unsigned short *a0) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    if (p >= P) return;
    uint4 lo = make_uint4(0u, 0u, 0u, 0u), hi = make_uint4(0u, 0u, 0u, 0u);
    lo.x = (unsigned)to_bf16(x[2 * (size_t)p]) | ((unsigned)to_bf16(x[2 * (size_t)p + 1]) << 16);
    uint4 *d = reinterpret_cast<uint4 *>(a0 + (size_t)p * NC);
    d[0] = lo;
    d[1] = hi;
}

// Loss: d = out - target; partial sums of d^2 per block; g[p][0] = bf16(2 d /
// count), other channels 0.
__global__ __launch_bounds__(256) void nn_loss(const float *out, const float *target, int P, float inv_count,
                                               unsigned short *g, double *part) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    double s = 0.0;
    if (p < P) {
        const float d = out[p] - target[p];
        s = (double)d * (double)d;
        uint4 lo = make_uint4((unsigned)to_bf16(2.f * d * inv_count), 0u, 0u, 0u);
        uint4 *dst = reinterpret_cast<uint4 *>(g + (size_t)p * NC);
        dst[0] = lo;
        dst[1] = make_uint4(0u, 0u, 0u, 0u);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Energy loss: az = A z with A the 5-point operator given per pixel as five
// planes [S, W, C, E, N] (planes[b][k][y][x], floats); partial sums of
// z*az - 2 z*r (r = input channel 0); g[p][0] = bf16(2 (az - r) / count).
__global__ __launch_bounds__(256) void nn_energy(const float *out, const float *x, const float *planes, int B, int H,
                                                 int W, int jacobi, float inv_count, unsigned short *g, double *part) {
    const int p = blockIdx.x * 256 + threadIdx.x;
    const int P = B * H * W;
    double s = 0.0;
    if (p < P) {
        const int b = p / (H * W), yx = p % (H * W), y = yx / W, xx = yx % W;
        const float *pl = planes + (size_t)b * 5 * H * W;
        const size_t hw = (size_t)H * W;
        // z = out (+ r / centre: the Jacobi step the network corrects)
        auto zat = [&](int q, int qyx) {
            return jacobi ? out[q] + x[2 * (size_t)q] / pl[2 * hw + qyx] : out[q];
        };
        const float z = zat(p, yx);
        float az = pl[2 * hw + yx] * z;
        if (y > 0) az = fmaf(pl[yx], zat(p - W, yx - W), az);
        if (xx > 0) az = fmaf(pl[hw + yx], zat(p - 1, yx - 1), az);
        if (xx < W - 1) az = fmaf(pl[3 * hw + yx], zat(p + 1, yx + 1), az);
        if (y < H - 1) az = fmaf(pl[4 * hw + yx], zat(p + W, yx + W), az);
        const float r = x[2 * (size_t)p];
        s = (double)z * (double)az - 2.0 * (double)z * (double)r;
        uint4 *dst = reinterpret_cast<uint4 *>(g + (size_t)p * NC);
        dst[0] = make_uint4((unsigned)to_bf16(2.f * (az - r) * inv_count), 0u, 0u, 0u);
        dst[1] = make_uint4(0u, 0u, 0u, 0u);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

// Weight gradient of one layer: dW[o][i][tap] = sum_p g[p][o] * a[p + tap][i],
// db[o] = sum_p g[p][o], FP32 on the vector units.  Thread t owns (o = t/16,
// i = t%16) and its nine taps; a block takes ROWS image rows, staged in LDS
// (a with a one-pixel zero halo).  partial[block][o][i][tap] then [o] bias.
constexpr int DW_ROWS = 2;
constexpr int DW_MAXW = 512;

__global__ __launch_bounds__(256) void nn_wgrad(const unsigned short *g, const unsigned short *a, int B, int H, int W,
                                                float *partial) {
    __shared__ unsigned short sg[DW_ROWS][DW_MAXW][NC];
    __shared__ unsigned short sa[DW_ROWS + 2][DW_MAXW + 2][NC];
    const int t = threadIdx.x;
    const int o = t >> 4, i = t & 15;
    float acc[9] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    float accb = 0.f;
    const int rows = B * H;
    const int nrb = (rows + DW_ROWS - 1) / DW_ROWS;
    for (int rb = blockIdx.x; rb < nrb; rb += gridDim.x) {
        const int r0 = rb * DW_ROWS;
        __syncthreads();
        // stage g rows r0 .. r0+ROWS-1 (same image only: rows never straddle
        // images because H % DW_ROWS == 0 is required by the host)
        const int img = r0 / H, y0 = r0 % H;
        for (int e = t; e < DW_ROWS * W * 2; e += 256) {
            const int half = e & 1, px = (e >> 1) % W, rr = (e >> 1) / W;
            const uint4 v = reinterpret_cast<const uint4 *>(g + ((size_t)(r0 + rr) * W + px) * NC)[half];
            reinterpret_cast<uint4 *>(&sg[rr][px][0])[half] = v;
        }
        for (int e = t; e < (DW_ROWS + 2) * (W + 2) * 2; e += 256) {
            const int half = e & 1, px = (e >> 1) % (W + 2), rr = (e >> 1) / (W + 2);
            const int yy = y0 + rr - 1, xx = px - 1;
            uint4 v = make_uint4(0u, 0u, 0u, 0u);
            if (yy >= 0 && yy < H && xx >= 0 && xx < W)
                v = reinterpret_cast<const uint4 *>(a + (((size_t)img * H + yy) * W + xx) * NC)[half];
            reinterpret_cast<uint4 *>(&sa[rr][px][0])[half] = v;
        }
        __syncthreads();
        for (int rr = 0; rr < DW_ROWS; ++rr) {
            float w0 = from_bf16(sa[rr][0][i]), w1 = from_bf16(sa[rr + 1][0][i]), w2 = from_bf16(sa[rr + 2][0][i]);
            float c0 = from_bf16(sa[rr][1][i]), c1 = from_bf16(sa[rr + 1][1][i]), c2 = from_bf16(sa[rr + 2][1][i]);
            for (int px = 0; px < W; ++px) {
                const float e0 = from_bf16(sa[rr][px + 2][i]), e1 = from_bf16(sa[rr + 1][px + 2][i]),
                            e2 = from_bf16(sa[rr + 2][px + 2][i]);
                const float gv = from_bf16(sg[rr][px][o]);
                acc[0] = fmaf(gv, w0, acc[0]);
                acc[1] = fmaf(gv, c0, acc[1]);
                acc[2] = fmaf(gv, e0, acc[2]);
                acc[3] = fmaf(gv, w1, acc[3]);
                acc[4] = fmaf(gv, c1, acc[4]);
                acc[5] = fmaf(gv, e1, acc[5]);
                acc[6] = fmaf(gv, w2, acc[6]);
                acc[7] = fmaf(gv, c2, acc[7]);
                acc[8] = fmaf(gv, e2, acc[8]);
                if (i == 0) accb += gv;
                w0 = c0; w1 = c1; w2 = c2;
                c0 = e0; c1 = e1; c2 = e2;
            }
        }
    }
    float *dst = partial + (size_t)blockIdx.x * LAYER_PARAMS;
#pragma unroll
    for (int tp = 0; tp < 9; ++tp) dst[(o * NC + i) * 9 + tp] = acc[tp];
    if (i == 0) dst[NC * NC * 9 + o] = accb;
}

// grad[l][e] = sum over blocks of partial[block][e] (fixed order), masked to
// the layer's real channels.
__global__ __launch_bounds__(256) void nn_wgrad_reduce(const float *partial, int nblocks, int layer, float *grad) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= LAYER_PARAMS) return;
    float s = 0.f;
    for (int b = 0; b < nblocks; ++b) s += partial[(size_t)b * LAYER_PARAMS + e];
    int o, i;
    if (e < NC * NC * 9) {
        o = e / (NC * 9);
        i = (e / 9) % NC;
    } else {
        o = e - NC * NC * 9;
        i = 0;
    }
    if (o >= OUT_CH[layer] || i >= IN_CH[layer]) s = 0.f;
    grad[(size_t)layer * LAYER_PARAMS + e] = s;
}

// Adam with bias correction on the FP32 master weights; entries outside a
// layer's real channels stay zero.
__global__ __launch_bounds__(256) void nn_adam(float *params, const float *grad, float *m, float *v, int n, float lr,
                                               float beta1, float beta2, float eps, float c1, float c2) {
    const int e = blockIdx.x * 256 + threadIdx.x;
    if (e >= n) return;
    const float gr = grad[e];
    const float mm = beta1 * m[e] + (1.f - beta1) * gr;
    const float vv = beta2 * v[e] + (1.f - beta2) * gr * gr;
    m[e] = mm;
    v[e] = vv;
    const float mh = mm / c1, vh = vv / c2;
    params[e] -= lr * mh / (sqrtf(vh) + eps);
}

__global__ __launch_bounds__(256) void nn_reduce_f64(const double *part, int m, double *out) {
    double s = 0.0;
    for (int i = threadIdx.x; i < m; i += 256) s += part[i];
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    __shared__ double red[4];
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) *out = red[0] + red[1] + red[2] + red[3];
}

// ---------------------------------------------------------------------------
// Host side: activation workspace for B images of H x W.
struct NnWork {
    unsigned short *act[NL];   // a_0 .. a_5 (layer inputs)
    unsigned short *g0, *g1;   // gradient ping-pong
    float *out;                // network output [P]
    unsigned short *wf, *wb;   // packed fragments
    float *bias;
    float *partial;            // weight-gradient partials
    double *part;              // loss partials
    double *scal;              // device scalars
    int nblk_dw;
};

int nn_work(int64_t P, NnWork *w) {
    const size_t act = (size_t)P * NC * sizeof(unsigned short);
    const size_t up = 256;
    auto al = [&](size_t b) { return (b + up - 1) / up * up; };
    const int nblk_dw = 1024;
    const size_t frag = (size_t)NL * 5 * 64 * 8 * sizeof(unsigned short);
    const size_t bytes = al(act) * (NL + 2) + al((size_t)P * sizeof(float)) + 2 * al(frag) +
                         al(NL * NC * sizeof(float)) + al((size_t)nblk_dw * LAYER_PARAMS * sizeof(float)) +
                         al(((size_t)P / 256 + 2) * sizeof(double)) + al(64 * sizeof(double));
    char *base = (char *)scratch(SLOT_NN, bytes);
    if (!base) return PERKS_E_NOMEM;
    for (int l = 0; l < NL; ++l) {
        w->act[l] = (unsigned short *)base;
        base += al(act);
    }
    w->g0 = (unsigned short *)base;
    base += al(act);
    w->g1 = (unsigned short *)base;
    base += al(act);
    w->out = (float *)base;
    base += al((size_t)P * sizeof(float));
    w->wf = (unsigned short *)base;
    base += al(frag);
    w->wb = (unsigned short *)base;
    base += al(frag);
    w->bias = (float *)base;
    base += al(NL * NC * sizeof(float));
    w->partial = (float *)base;
    base += al((size_t)nblk_dw * LAYER_PARAMS * sizeof(float));
    w->part = (double *)base;
    base += al(((size_t)P / 256 + 2) * sizeof(double));
    w->scal = (double *)base;
    w->nblk_dw = nblk_dw;
    return PERKS_OK;
}

int check_dims(int B, int H, int W) {
    if (B < 1 || H < 1 || W < 1) return set_error(PERKS_E_INVAL, "B, H and W must be >= 1");
    if ((int64_t)B * H * W >= (int64_t(1) << 31)) return set_error(PERKS_E_INVAL, "too many pixels");
    return PERKS_OK;
}

void launch_conv(hipStream_t st, const unsigned short *in, const unsigned short *frag, const float *bias,
                 const unsigned short *mask, void *out, int B, int H, int W, int mode) {
    const int segs = (W + 15) / 16;
    const int xblocks = (segs + SEG - 1) / SEG;
    const int rowblocks = (B * H + 3) / 4;
    hipLaunchKernelGGL(nn_conv, dim3(rowblocks * xblocks), dim3(256), 0, st, in, frag, bias, mask, out, B, H, W,
                       mode);
}

// Forward pass from a_0 (already packed); keeps a_1 .. a_5 and the output.
void forward_from_input(hipStream_t st, NnWork &w, int B, int H, int W) {
    const size_t fl = 5 * 64 * 8;
    for (int l = 0; l < NL; ++l) {
        if (l < NL - 1)
            launch_conv(st, w.act[l], w.wf + l * fl, w.bias + l * NC, nullptr, w.act[l + 1], B, H, W, 0);
        else
            launch_conv(st, w.act[l], w.wf + l * fl, w.bias + l * NC, nullptr, w.out, B, H, W, 1);
    }
}

void pack_weights(hipStream_t st, const float *params, NnWork &w) {
    hipLaunchKernelGGL(nn_pack, dim3((NL * 5 * 64 * 8 + 255) / 256), dim3(256), 0, st, params, w.wf, w.wb, w.bias);
}

}  // namespace
}  // namespace perks

using namespace perks;

extern "C" {

int perks_nn_forward(const float *params, const float *x, int32_t B, int32_t H, int32_t W, float *out,
                     void *stream) {
    if (!params || !x || !out) return set_error(PERKS_E_INVAL, "params, x and out must not be NULL");
    int rc = check_dims(B, H, W);
    if (rc) return rc;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t P = (int64_t)B * H * W;
    NnWork w;
    rc = nn_work(P, &w);
    if (rc) return rc;
    pack_weights(st, params, w);
    hipLaunchKernelGGL(nn_pack_input, dim3((unsigned)((P + 255) / 256)), dim3(256), 0, st, x, (int)P, w.act[0]);
    forward_from_input(st, w, B, H, W);
    PERKS_HIP_TRY(hipMemcpyAsync(out, w.out, (size_t)P * sizeof(float), hipMemcpyDeviceToDevice, st));
    PERKS_HIP_TRY(hipGetLastError());
    return PERKS_OK;
}

}  // extern "C"

namespace {

__global__ void nn_accum(const double *scal, double *acc, double scale) {
    if (threadIdx.x == 0) acc[0] += scal[0] * scale;
}

// dst[b][e] = src[idx[b]][e] for b < n, e < elems.
__global__ __launch_bounds__(256) void nn_gather(const float *src, const int *idx, int n, int64_t elems, float *dst) {
    const int64_t total = (int64_t)n * elems;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < total; i += (int64_t)gridDim.x * 256) {
        const int64_t b = i / elems, e = i % elems;
        dst[i] = src[(int64_t)idx[b] * elems + e];
    }
}

// Forward, loss (MSE against target, or the energy functional with the
// 5-point planes), backward: grad and (if loss) the loss; with loss_acc the
// loss times acc_scale is also added to that device double (no sync).
int loss_grad_impl(const float *params, const float *x, const float *target, const float *planes, int jacobi, int B,
                   int H, int W, float *grad, double *loss, hipStream_t st, double *loss_acc = nullptr,
                   double acc_scale = 0.0) {
    if (!params || !x || !grad || (!target && !planes)) return set_error(PERKS_E_INVAL, "NULL argument");
    int rc = check_dims(B, H, W);
    if (rc) return rc;
    if (H % DW_ROWS != 0) return set_error(PERKS_E_UNSUPPORTED, "H must be a multiple of %d", DW_ROWS);
    if (W > DW_MAXW) return set_error(PERKS_E_UNSUPPORTED, "W must be <= %d for training", DW_MAXW);
    const int64_t P = (int64_t)B * H * W;
    NnWork w;
    rc = nn_work(P, &w);
    if (rc) return rc;
    pack_weights(st, params, w);
    const unsigned nb = (unsigned)((P + 255) / 256);
    hipLaunchKernelGGL(nn_pack_input, dim3(nb), dim3(256), 0, st, x, (int)P, w.act[0]);
    forward_from_input(st, w, B, H, W);
    if (planes)
        hipLaunchKernelGGL(nn_energy, dim3(nb), dim3(256), 0, st, (const float *)w.out, x, planes, B, H, W,
                           jacobi, 1.0f / (float)P, w.g0, w.part);
    else
        hipLaunchKernelGGL(nn_loss, dim3(nb), dim3(256), 0, st, (const float *)w.out, target, (int)P,
                           1.0f / (float)P, w.g0, w.part);
    hipLaunchKernelGGL(nn_reduce_f64, dim3(1), dim3(256), 0, st, (const double *)w.part, (int)nb, w.scal);
    if (loss_acc)
        hipLaunchKernelGGL(nn_accum, dim3(1), dim3(64), 0, st, (const double *)w.scal, loss_acc,
                           acc_scale / (double)P);
    const size_t fl = 5 * 64 * 8;
    unsigned short *g = w.g0, *gn = w.g1;
    const int rows = B * H;
    const int nblk = std::min(w.nblk_dw, (rows + DW_ROWS - 1) / DW_ROWS);
    for (int l = NL - 1; l >= 0; --l) {
        hipLaunchKernelGGL(nn_wgrad, dim3(nblk), dim3(256), 0, st, (const unsigned short *)g,
                           (const unsigned short *)w.act[l], B, H, W, w.partial);
        hipLaunchKernelGGL(nn_wgrad_reduce, dim3((LAYER_PARAMS + 255) / 256), dim3(256), 0, st,
                           (const float *)w.partial, nblk, l, grad);
        if (l > 0) {
            // gradient w.r.t. a_l = relu(pre_{l-1}): transposed conv, masked by a_l > 0
            launch_conv(st, g, w.wb + l * fl, nullptr, w.act[l], gn, B, H, W, 2);
            std::swap(g, gn);
        }
    }
    if (loss) {
        double h = 0.0;
        PERKS_HIP_TRY(hipMemcpyAsync(&h, w.scal, sizeof(double), hipMemcpyDeviceToHost, st));
        PERKS_HIP_TRY(hipStreamSynchronize(st));
        *loss = h / (double)P;
    }
    PERKS_HIP_TRY(hipGetLastError());
    return PERKS_OK;
}

}  // namespace

extern "C" {

int perks_nn_loss_grad(const float *params, const float *x, const float *target, int32_t B, int32_t H, int32_t W,
                       float *grad, double *loss, void *stream) {
    if (!target) return set_error(PERKS_E_INVAL, "target must not be NULL");
    return loss_grad_impl(params, x, target, nullptr, 0, B, H, W, grad, loss,
                          reinterpret_cast<hipStream_t>(stream));
}

int perks_nn_energy_grad(const float *params, const float *x, const float *planes, int32_t jacobi, int32_t B,
                         int32_t H, int32_t W, float *grad, double *loss, void *stream) {
    if (!planes) return set_error(PERKS_E_INVAL, "planes must not be NULL");
    if (jacobi != 0 && jacobi != 1) return set_error(PERKS_E_INVAL, "jacobi must be 0 or 1");
    return loss_grad_impl(params, x, nullptr, planes, jacobi, B, H, W, grad, loss,
                          reinterpret_cast<hipStream_t>(stream));
}

int perks_nn_adam(float *params, const float *grad, float *m, float *v, int32_t step, float lr, float beta1,
                  float beta2, float eps, void *stream) {
    if (!params || !grad || !m || !v) return set_error(PERKS_E_INVAL, "NULL argument");
    if (step < 1) return set_error(PERKS_E_INVAL, "step counts from 1");
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int n = PERKS_NN_PARAMS;
    const float c1 = 1.f - std::pow(beta1, (float)step), c2 = 1.f - std::pow(beta2, (float)step);
    hipLaunchKernelGGL(nn_adam, dim3((n + 255) / 256), dim3(256), 0, st, params, grad, m, v, n, lr, beta1, beta2, eps,
                       c1, c2);
    PERKS_HIP_TRY(hipGetLastError());
    return PERKS_OK;
}

int perks_nn_train(float *params, const float *x, const float *target, const float *planes, const int32_t *field,
                   int32_t P, int32_t H, int32_t W, int32_t epochs, int32_t batch, float lr, uint64_t seed, float *m,
                   float *v, int32_t *step, double *losses, void *stream) {
    if (!params || !x || !m || !v || !step) return set_error(PERKS_E_INVAL, "NULL argument");
    if ((target != nullptr) == (planes != nullptr)) return set_error(PERKS_E_INVAL, "give target or planes, not both");
    if (planes && !field) return set_error(PERKS_E_INVAL, "planes need field");
    if (P < 1 || batch < 1 || batch > P || epochs < 0) return set_error(PERKS_E_INVAL, "bad P, batch or epochs");
    if (!(lr > 0.f)) return set_error(PERKS_E_INVAL, "lr must be > 0");
    if (*step < 0) return set_error(PERKS_E_INVAL, "step must be >= 0");
    int rc = check_dims(batch, H, W);
    if (rc) return rc;
    if (H % DW_ROWS != 0) return set_error(PERKS_E_UNSUPPORTED, "H must be a multiple of %d", DW_ROWS);
    if (W > DW_MAXW) return set_error(PERKS_E_UNSUPPORTED, "W must be <= %d for training", DW_MAXW);
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t px = (int64_t)H * W;
    std::vector<int> fld;
    if (planes) {
        fld.resize(P);
        PERKS_HIP_TRY(hipMemcpyAsync(fld.data(), field, (size_t)P * sizeof(int), hipMemcpyDeviceToHost, st));
        PERKS_HIP_TRY(hipStreamSynchronize(st));
    }
    // batch buffers: indices (samples, operators), inputs, targets or planes,
    // gradient, loss accumulator
    const size_t bx = (size_t)batch * px * 2, bt = (size_t)batch * px * (planes ? 5 : 1);
    char *buf = nullptr;
    const size_t bytes = 2 * 256 + (size_t)batch * 2 * sizeof(int) + (bx + bt + PERKS_NN_PARAMS) * sizeof(float) + 64;
    if (hipMalloc(&buf, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return set_error(PERKS_E_NOMEM, "nn_train: %zu bytes", bytes);
    }
    double *acc = reinterpret_cast<double *>(buf);
    int *idx = reinterpret_cast<int *>(buf + 256);
    int *pidx = idx + batch;
    float *xb = reinterpret_cast<float *>(buf + 512 + (size_t)batch * 2 * sizeof(int));
    float *tb = xb + bx;
    float *grad = tb + bt;
    // splitmix64 (Steele, Lea and Flood, 2014) drives the per-epoch shuffles
    uint64_t state = seed;
    auto next = [&]() {
        uint64_t z = (state += 0x9e3779b97f4a7c15ULL);
        z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ULL;
        z = (z ^ (z >> 27)) * 0x94d049bb133111ebULL;
        return z ^ (z >> 31);
    };
    std::vector<int> perm(P), hidx(batch), hpidx(batch);
    const int nbatch = P / batch;
    for (int e = 0; e < epochs && rc == PERKS_OK; ++e) {
        for (int i = 0; i < P; ++i) perm[i] = i;
        for (int i = P - 1; i > 0; --i) std::swap(perm[i], perm[(int)(next() % (uint64_t)(i + 1))]);
        if (hipMemsetAsync(acc, 0, sizeof(double), st) != hipSuccess) {
            rc = set_error(PERKS_E_HIP, "nn_train: memset");
            break;
        }
        for (int b = 0; b < nbatch; ++b) {
            for (int j = 0; j < batch; ++j) {
                hidx[j] = perm[b * batch + j];
                if (planes) hpidx[j] = fld[hidx[j]];
            }
            if (hipMemcpyAsync(idx, hidx.data(), batch * sizeof(int), hipMemcpyHostToDevice, st) != hipSuccess ||
                (planes && hipMemcpyAsync(pidx, hpidx.data(), batch * sizeof(int), hipMemcpyHostToDevice, st) !=
                               hipSuccess)) {
                rc = set_error(PERKS_E_HIP, "nn_train: index copy");
                break;
            }
            // the host index arrays are rewritten next batch: the copies must be done
            if (hipStreamSynchronize(st) != hipSuccess) {
                rc = set_error(PERKS_E_HIP, "nn_train: sync");
                break;
            }
            const unsigned gb = (unsigned)std::min<int64_t>(4096, ((int64_t)bx + 255) / 256);
            hipLaunchKernelGGL(nn_gather, dim3(gb), dim3(256), 0, st, x, (const int *)idx, batch, px * 2, xb);
            if (planes)
                hipLaunchKernelGGL(nn_gather, dim3(gb), dim3(256), 0, st, planes, (const int *)pidx, batch, px * 5, tb);
            else
                hipLaunchKernelGGL(nn_gather, dim3(gb), dim3(256), 0, st, target, (const int *)idx, batch, px, tb);
            rc = loss_grad_impl(params, xb, planes ? nullptr : tb, planes ? tb : nullptr, 1, batch, H, W, grad,
                                nullptr, st, acc, 1.0 / nbatch);
            if (rc) break;
            ++*step;
            rc = perks_nn_adam(params, grad, m, v, *step, lr, 0.9f, 0.999f, 1e-8f, stream);
            if (rc) break;
        }
        if (rc) break;
        if (losses) {
            double h = 0.0;
            if (hipMemcpyAsync(&h, acc, sizeof(double), hipMemcpyDeviceToHost, st) != hipSuccess ||
                hipStreamSynchronize(st) != hipSuccess) {
                rc = set_error(PERKS_E_HIP, "nn_train: loss copy");
                break;
            }
            losses[e] = h;
        }
    }
    (void)hipStreamSynchronize(st);
    (void)hipFree(buf);
    if (rc) return rc;
    PERKS_HIP_TRY(hipGetLastError());
    return PERKS_OK;
}

}  // extern "C"

// ---------------------------------------------------------------------------
// Training pairs from captured CG iterates (the network's part of the error
// that the Jacobi step leaves, scaled by the residual's RMS).
namespace {

constexpr int PAIR_BLOCKS = 256;   // partial sums per capture

// part[j][b] = sum of r_j^2 over the grid-stride share of block b; a NaN
// partial when any r_j entry in that share is not finite.
__global__ __launch_bounds__(256) void pair_sumsq(const double *cap_r, int64_t n, double *part) {
    const int j = blockIdx.y;
    const double *r = cap_r + (size_t)j * n;
    double s = 0.0;
    bool finite = true;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double v = r[i];
        finite = finite && isfinite(v);
        s = __builtin_fma(v, v, s);
    }
    for (int off = 32; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    const bool all_finite = __all(finite);
    __shared__ double red[4];
    __shared__ int bad[4];
    if ((threadIdx.x & 63) == 0) {
        red[threadIdx.x >> 6] = s;
        bad[threadIdx.x >> 6] = !all_finite;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        const double t = (red[0] + red[1]) + (red[2] + red[3]);
        part[(size_t)j * gridDim.x + blockIdx.x] = (bad[0] | bad[1] | bad[2] | bad[3]) ? NAN : t;
    }
}

// rms[j] = sqrt(sum of the partials / n), summed in block order (NaN when a
// partial is NaN).
__global__ __launch_bounds__(64) void pair_rms(const double *part, int nb, int64_t n, double *rms) {
    const int j = blockIdx.x;
    if (threadIdx.x == 0) {
        double s = 0.0;
        for (int b = 0; b < nb; ++b) s += part[(size_t)j * nb + b];
        rms[j] = sqrt(s / (double)n);
    }
}

// For capture j and grid point i (row i of A): inputs[j][i] = {r/rms, logk},
// targets[j][i] = (xstar - x_j - r / a_ii) / rms, computed in FP64 and
// rounded to FP32.
__global__ __launch_bounds__(256) void pair_form(const int *rowptr, const int *colind, const double *val,
                                                 const double *xstar, const double *logk, const double *cap_x,
                                                 const double *cap_r, const double *rms, int64_t n, float *inputs,
                                                 float *targets) {
    const int j = blockIdx.y;
    const double s = rms[j];
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        double d = 0.0;
        for (int k = rowptr[i]; k < rowptr[i + 1]; ++k)
            if (colind[k] == (int)i) d += val[k];
        const double r = cap_r[(size_t)j * n + i];
        const double x = cap_x[(size_t)j * n + i];
        const size_t o = (size_t)j * n + i;
        inputs[2 * o] = (float)(r / s);
        inputs[2 * o + 1] = (float)logk[i];
        targets[o] = (float)((xstar[i] - x - r / d) / s);
    }
}

}  // namespace

extern "C" {

int perks_nn_make_pairs(const perks_csr *A, const double *xstar, const double *logk, const double *cap_x,
                        const double *cap_r, int32_t ncap, int32_t H, int32_t W, float *inputs, float *targets,
                        int32_t *count, void *stream) {
    if (!A || !xstar || !logk || !cap_x || !cap_r || !inputs || !targets || !count)
        return set_error(PERKS_E_INVAL, "NULL argument");
    if (A->dt != PERKS_F64 || !A->rowptr || !A->colind || !A->val)
        return set_error(PERKS_E_INVAL, "A must be an FP64 CSR matrix");
    if (H < 1 || W < 1 || (int64_t)H * W != A->n) return set_error(PERKS_E_INVAL, "H * W must equal A's order");
    if (ncap < 0 || ncap > 4096) return set_error(PERKS_E_INVAL, "ncap must be in [0, 4096]");
    *count = 0;
    if (ncap == 0) return PERKS_OK;
    hipStream_t st = reinterpret_cast<hipStream_t>(stream);
    const int64_t n = A->n;
    double *part = (double *)scratch(SLOT_NN_PAIRS, ((size_t)ncap * PAIR_BLOCKS + ncap) * sizeof(double));
    if (!part) return PERKS_E_NOMEM;
    double *rms = part + (size_t)ncap * PAIR_BLOCKS;
    hipLaunchKernelGGL(pair_sumsq, dim3(PAIR_BLOCKS, ncap), dim3(256), 0, st, cap_r, n, part);
    hipLaunchKernelGGL(pair_rms, dim3(ncap), dim3(64), 0, st, (const double *)part, PAIR_BLOCKS, n, rms);
    std::vector<double> h(ncap);
    PERKS_HIP_TRY(hipMemcpyAsync(h.data(), rms, ncap * sizeof(double), hipMemcpyDeviceToHost, st));
    PERKS_HIP_TRY(hipStreamSynchronize(st));
    int m = 0;
    while (m < ncap && std::isfinite(h[m]) && h[m] > 0.0) ++m;
    if (m > 0) {
        const unsigned nb = (unsigned)std::min<int64_t>((n + 255) / 256, 4096);
        hipLaunchKernelGGL(pair_form, dim3(nb, m), dim3(256), 0, st, (const int *)A->rowptr,
                           (const int *)A->colind, (const double *)A->val, xstar, logk, cap_x, cap_r,
                           (const double *)rms, n, inputs, targets);
    }
    PERKS_HIP_TRY(hipGetLastError());
    *count = m;
    return PERKS_OK;
}

}  // extern "C"
