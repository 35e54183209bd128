// Launch interface of the surrogate's BF16/FP32 kernels (unet_kernels.hip).
// Tensors are NHWC; 3x3 weights are W[co][tap][ci] with tap = 3*dy + dx.
#pragma once

#include <hip/hip_runtime.h>

namespace rlbm {

// out = act(conv3x3(in, w) + bias), zero padding, BF16 in/out, FP32 accumulation (Ci, Co multiples of 16).
hipError_t conv3x3_forward(const void *in, const void *w, const float *bias, void *out, int B, int H, int W, int Ci,
                           int Co, bool relu, hipStream_t s);
// The input and the optional extra outputs of a forward convolution.
struct ConvInputs {
    const void *in = nullptr;    // B x H x W x Ci; with skip: B x H/2 x W/2 x cu, upsampled 2x (nearest)
    const void *skip = nullptr;  // with skip, the input is [up(in) | skip], skip B x H x W x (Ci - cu)
    int cu = 0;
    void *pooled = nullptr;      // also write the 2x2 average of the output, B x H/2 x W/2 x Co
    const void *head_w = nullptr;  // also apply a 1x1 head (BF16 head_o x Co weights, FP32 bias) to the output
    const float *head_b = nullptr;
    float *head_out = nullptr;   // B x H x W x head_o, FP32
    int head_o = 0;
};
hipError_t conv3x3_forward_ex(const ConvInputs &x, const void *w, const float *bias, void *out, int B, int H, int W,
                              int Ci, int Co, bool relu, hipStream_t s);
// wt[ci][8 - tap][co] = w[co][tap][ci]; the gradient with respect to the input of a 3x3
// convolution is conv3x3_forward(dout, wt) (no bias, no activation).
hipError_t conv3x3_adjoint_weights(const void *w, void *wt, int Ci, int Co, hipStream_t s);
// The same for up to kMaxAdjoint layers in one launch: layer k's weights at
// element w + woff[k] (Co x 9 x Ci) go transposed to element wt + toff[k];
// the layers lie back to back in wt (toff[k + 1] = toff[k] + Co 9 Ci).
constexpr int kMaxAdjoint = 32;
struct AdjointTable {
    int n;
    long long woff[kMaxAdjoint], toff[kMaxAdjoint + 1];
    int ci[kMaxAdjoint], co[kMaxAdjoint];
};
hipError_t conv3x3_adjoint_weights_all(const void *w, void *wt, const AdjointTable &t, hipStream_t s);
// Weight-gradient partials (chunks of whole image rows); part needs
// conv3x3_wgrad_chunks(B, H, W, Ci, Co) * Co * 9 * Ci floats.
int conv3x3_wgrad_chunks(int B, int H, int W, int Ci, int Co);
// gw[co][tap][ci] += sum_p dpre[p][co] * in[p + tap][ci] (deterministic two-pass reduction through part).
hipError_t conv3x3_backward_weight(const void *dpre, const void *in, float *part, float *gw, int B, int H, int W,
                                   int Ci, int Co, hipStream_t s);
// The weight-gradient partials alone (the reduction left to reduce_partials);
// returns the number of chunks written to part, or -1 on a launch error.
int conv3x3_backward_weight_part(const void *dpre, const void *in, float *part, int B, int H, int W, int Ci, int Co,
                                 hipStream_t s);
// Deferred reductions: job j adds sum over c < chunks[j] of
// part[j][c * len[j] + q] to g[j][q] for q < len[j] (a fixed order:
// deterministic); all jobs in one launch.
constexpr int kMaxReduceJobs = 48;
struct ReduceJobs {
    int n = 0;
    long long block_start[kMaxReduceJobs + 1] = {};
    const float *part[kMaxReduceJobs] = {};
    float *g[kMaxReduceJobs] = {};
    long long len[kMaxReduceJobs] = {};
    int chunks[kMaxReduceJobs] = {};
};
// Appends a job (false when the table is full).
bool add_reduce_job(ReduceJobs &j, const float *part, float *g, long long len, int chunks);
hipError_t reduce_partials(const ReduceJobs &j, hipStream_t s);
// Blocks of the per-channel and head-gradient sums: part needs
// channel_sum_blocks(npix) * C floats (head_backward: * O * (C + 1)).
constexpr int kSumBlocks = 512;
int channel_sum_blocks(long long npix);
// gb[c] += sum_p d[p][c] (deterministic two-pass sum through part when C
// divides 256, one block per channel otherwise)
hipError_t channel_sum(const void *d, float *part, float *gb, long long npix, int C, hipStream_t s);
// d *= (out > 0)
hipError_t relu_backward(void *d, const void *out, long long n, hipStream_t s);
// d *= (out > 0) over npix x C and gb[c] += sum_p d[p][c], in one pass when
// C % 8 == 0 and C / 8 divides 256 (part as for channel_sum)
hipError_t relu_backward_bias(void *d, const void *out, float *part, float *gb, long long npix, int C, hipStream_t s);
// The same with the bias sums left as channel_sum_blocks(npix) rows of C
// partials in part (for reduce_partials) when C % 8 == 0 and C / 8 divides
// 256 (*rows = the row count); otherwise as relu_backward_bias (*rows = 0).
hipError_t relu_backward_bias_part(void *d, const void *out, float *part, float *gb, long long npix, int C, int *rows,
                                   hipStream_t s);
hipError_t pool_forward(const void *in, void *out, int B, int H, int W, int C, hipStream_t s);
// dx = dy / 4 broadcast to 2x2 blocks (+ channels [skip_off, skip_off + C) of skip, a B*H*W*skip_c tensor)
hipError_t pool_backward(const void *dy, const void *skip, int skip_c, int skip_off, void *dx, int B, int H, int W,
                         int C, hipStream_t s);
hipError_t up_concat(const void *u, const void *skip, void *cat, int B, int H, int W, int Cu, int Cs, hipStream_t s);
hipError_t up_backward(const void *dcat, void *du, int B, int H, int W, int Cu, int C, hipStream_t s);
hipError_t head_forward(const void *x, const void *w, const float *b, float *y, long long npix, int C, int O,
                        hipStream_t s);
// Head (1x1, C = 16 -> O = 3) backward: dx, and gw, gb += the parameter
// gradients (deterministic two-pass sums through part).
hipError_t head_backward(const float *dy, const void *x, const void *w, void *dx, float *part, float *gw, float *gb,
                         long long npix, int C, int O, hipStream_t s);
hipError_t mse(const float *y, const float *t, float *dy, double *part, int nblocks, long long n, hipStream_t s);
hipError_t adam(float *theta, const float *g, float *m, float *v, void *theta_bf, long long n, float lr, float b1,
                float b2, float eps, float c1, float c2, hipStream_t s);
hipError_t to_bf16(const float *a, void *b, long long n, hipStream_t s);
hipError_t to_f32(const void *a, float *b, long long n, hipStream_t s);

}  // namespace rlbm
