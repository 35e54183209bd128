// gfx950 kernels of the convolutional warm-start surrogate (a U-Net):
// BF16 activations and weights, FP32 accumulation on the matrix cores.
//
// Layout: activations NHWC (channels innermost), 3x3 weights W[co][tap][ci]
// with tap = 3*dy + dx.  A 3x3 convolution is an implicit GEMM
//   out[pixel, co] = sum_{tap, ci} in[pixel + tap, ci] * W[co, tap, ci]
// with M = pixels, N = output channels, K = 9 * input channels.  Each
// wavefront owns a 16-pixel x 16-channel output tile and walks K in steps of
// 32 (v_mfma_f32_16x16x32_bf16) or 16 (v_mfma_f32_16x16x16_bf16) channels;
// each lane loads its 8 (or 4) consecutive channels of one pixel and of one
// weight row with a single vector load.  Operand layout of the 16x16xK
// matrix instruction (wave64): A[i][k] in lane i + 16*(k / (K/4)), element
// k % (K/4); B[k][j] likewise with j; C[i][j] in lane j + 16*(i/4), element
// i % 4.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdint>

#include "unet_kernels.h"

namespace rlbm {
namespace {

typedef __bf16 bf16;
typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float f32x4;

// ---------------------------------------------------------------- conv 3x3

// Geometry of one forward-convolution launch, computed on the host.  A
// block computes a patch of 64 * ROWS pixels of one image -- pr rows of pw
// pixels, pw = 64, or 32 or 16 when the image is that narrow -- for NB
// output channels.
struct ConvGeom {
    int H, W, Ci, Co;
    int pw_log2;        // log2 of the patch width pw
    int xw;             // staged row length, pw + 2 (one halo pixel each side)
    unsigned xw_magic;  // floor(2^32 / xw) + 1: p / xw == umulhi(p, xw_magic) for p < 2^16
    int patches_x, patches_y;
    int relu;
    int cu;      // input channels read from `in` (Ci, or the upsampled part of a concatenation)
    int head_o;  // outputs of a fused 1x1 head (0: none)
};

// out[p][co] = act(bias[co] + sum_{tap, ci} in[p + tap][ci] W[co][tap][ci]).
// grid.x = B * patches_y * patches_x, grid.y = Co / NB, 4 wavefronts.
//
// Input.  The input channels are taken CC at a time (a chunk): the block
// stages the chunk's (pr + 2) x (pw + 2) input pixels (zero outside the
// image) and its NB x 9 x CC weights through LDS.  Every 16-byte global load
// of a chunk is issued before the first LDS write, and the next chunk's loads
// are in flight while the matrix instructions consume the current one.  With
// CAT the input is the concatenation [nearest 2x upsampling of in | skip]
// (in: H/2 x W/2 x cu, skip: H x W x (Ci - cu)), read in place: a chunk lies
// wholly in one of the two.
//
// Product.  The K dimension of a chunk, 9 taps x CC channels, is walked 32 at
// a time with v_mfma_f32_16x16x32_bf16 (for CC = 16 a step spans two taps;
// the last step's missing tenth tap has zero weights).  Wavefront w owns the
// 16-pixel groups w, w + 4, ... of the patch and all NB channels: per step it
// reads ROWS pixel fragments and NB / 16 weight fragments and issues
// ROWS * NB / 16 matrix instructions.  The weights are the A operand, so a
// lane's accumulator holds 4 consecutive output channels of one pixel.
//
// Output.  The activated tile goes through LDS (BF16, as stored) and leaves
// in 16-byte stores; from the same tile the block can also write the 2x2
// average of its output (pooled: H/2 x W/2 x Co; pr and pw even) and a 1x1
// head (head_out[p][o] = head_b[o] + sum_c out[p][c] head_w[o][c], FP32;
// NB == Co).
template <int ROWS, int NB, int CC, bool CAT>
__global__ __launch_bounds__(256) void conv3x3_fwd_kernel(const bf16 *__restrict__ in, const bf16 *__restrict__ skip,
                                                          const bf16 *__restrict__ w, const float *__restrict__ bias,
                                                          bf16 *__restrict__ out, bf16 *__restrict__ pooled,
                                                          const bf16 *__restrict__ head_w,
                                                          const float *__restrict__ head_b, float *__restrict__ head_out,
                                                          const ConvGeom g)
{
    constexpr int G = CC / 8;                   // 16-byte groups per staged pixel
    constexpr int CP = CC + 8;                  // staged pixel stride (16 bytes of padding: no bank conflicts)
    constexpr int XPIX = (ROWS + 2) * 66;       // staged pixels of the widest patch shape (the most)
    constexpr int NS = (9 * CC + 31) / 32;      // K steps of 32 per chunk
    constexpr int WS = 32 * NS + 8;             // staged weight row of one output channel, padded
    constexpr int NT = NB / 16;                 // 16-channel output tiles
    constexpr int XU = (XPIX * G + 255) / 256;  // 16-byte staging units per thread
    constexpr int WU = (NB * 9 * G + 255) / 256;
    constexpr int TS = NB + 8;                  // output tile row (one pixel), padded
    static_assert(64 * ROWS * TS <= XPIX * CP + NB * WS, "the output tile reuses the staging LDS");
    __shared__ __attribute__((aligned(16))) bf16 smem[XPIX * CP + NB * WS];
    bf16 *const Xs = smem;
    bf16 *const Ws = smem + XPIX * CP;

    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int r = lane & 15, kq = lane >> 4;
    const int pw = 1 << g.pw_log2, pr = (64 * ROWS) >> g.pw_log2;
    int q = blockIdx.x;
    const int px0 = (q % g.patches_x) << g.pw_log2;
    q /= g.patches_x;
    const int py0 = (q % g.patches_y) * pr;
    const int b = q / g.patches_y;
    const int co0 = blockIdx.y * NB;
    const int xunits = (pr + 2) * g.xw * G;
    bf16x8 zero;
#pragma unroll
    for (int e = 0; e < 8; ++e) zero[e] = (bf16)0.f;

    // Staging loads are raw buffer loads: an offset past the end of the
    // buffer reads zero, which gives the zero padding outside the image and
    // idle units without branches around the loads.  Byte offsets of each
    // unit at channel 0 (kOut when the unit reads nothing), fixed for the block.
    constexpr unsigned kOut = 0x80000000u;
    const int hs = CAT ? 1 : 0;  // `in` is at half resolution in a concatenation
    const int cs = g.Ci - g.cu;
    const __amdgpu_buffer_rsrc_t xrs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(in + (long long)b * (g.H >> hs) * (g.W >> hs) * g.cu), (short)0,
        (g.H >> hs) * (g.W >> hs) * g.cu * 2, 0x00020000);
    const __amdgpu_buffer_rsrc_t srs = __builtin_amdgcn_make_buffer_rsrc(
        (void *)(CAT ? skip + (long long)b * g.H * g.W * cs : in), (short)0, CAT ? g.H * g.W * cs * 2 : 0, 0x00020000);
    const __amdgpu_buffer_rsrc_t wrs =
        __builtin_amdgcn_make_buffer_rsrc((void *)(w + (long long)co0 * 9 * g.Ci), (short)0, NB * 9 * g.Ci * 2, 0x00020000);
    unsigned xo[XU], so[CAT ? XU : 1], wo[WU];
#pragma unroll
    for (int i = 0; i < XU; ++i) {
        const int u = t + 256 * i;
        const unsigned p = (unsigned)u / G;
        const int row = (int)__umulhi(p, g.xw_magic);
        const int yy = py0 - 1 + row, xx = px0 - 1 + ((int)p - row * g.xw);
        const bool in_img = u < xunits && (unsigned)yy < (unsigned)g.H && (unsigned)xx < (unsigned)g.W;
        if constexpr (CAT) {
            xo[i] = in_img ? (unsigned)((((yy >> 1) * (g.W >> 1) + (xx >> 1)) * g.cu + 8 * (u % G)) * 2) : kOut;
            so[i] = in_img ? (unsigned)(((yy * g.W + xx) * cs + 8 * (u % G)) * 2) : kOut;
        } else {
            xo[i] = in_img ? (unsigned)(((yy * g.W + xx) * g.Ci + 8 * (u % G)) * 2) : kOut;
        }
    }
#pragma unroll
    for (int i = 0; i < WU; ++i) {
        const int u = t + 256 * i;  // u / G = co * 9 + tap
        wo[i] = u < NB * 9 * G ? (unsigned)(((u / G) * g.Ci + 8 * (u % G)) * 2) : kOut;
    }
    bf16x8 xr[XU], wr[WU];
    auto load = [&](int c0) {
        if constexpr (CAT) {
            const bool fu = c0 < g.cu;  // the whole chunk comes from one source
            const __amdgpu_buffer_rsrc_t rs = fu ? xrs : srs;
            const unsigned add = 2 * (fu ? c0 : c0 - g.cu);
#pragma unroll
            for (int i = 0; i < XU; ++i)
                xr[i] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(rs, (int)((fu ? xo[i] : so[i]) + add), 0, 0));
        } else {
#pragma unroll
            for (int i = 0; i < XU; ++i)
                xr[i] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(xrs, (int)(xo[i] + 2 * c0), 0, 0));
        }
#pragma unroll
        for (int i = 0; i < WU; ++i)
            wr[i] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(wrs, (int)(wo[i] + 2 * c0), 0, 0));
    };
    auto stage = [&]() {
#pragma unroll
        for (int i = 0; i < XU; ++i) {
            const int u = t + 256 * i;
            if ((XPIX * G) % 256 == 0 || u < XPIX * G) *reinterpret_cast<bf16x8 *>(&Xs[(u / G) * CP + 8 * (u % G)]) = xr[i];
        }
#pragma unroll
        for (int i = 0; i < WU; ++i) {
            const int u = t + 256 * i;
            if ((NB * 9 * G) % 256 == 0 || u < NB * 9 * G) {
                const int k = u / G, co = k / 9, tap = k - 9 * co;
                *reinterpret_cast<bf16x8 *>(&Ws[co * WS + tap * CC + 8 * (u % G)]) = wr[i];
            }
        }
    };
    // zero weights for the padding of the last K step (CC = 16 only); never overwritten
    if constexpr (32 * NS > 9 * CC) {
        constexpr int PADG = (32 * NS - 9 * CC) / 8;
        for (int u = t; u < NB * PADG; u += 256)
            *reinterpret_cast<bf16x8 *>(&Ws[(u / PADG) * WS + 9 * CC + 8 * (u % PADG)]) = zero;
    }
    // per-lane LDS offsets: the lane's pixel in each of its groups, and the
    // (tap, channel) of its 8 K values in each step (the padding tap reads tap 8)
    int xoff[ROWS], toff[NS];
#pragma unroll
    for (int rr = 0; rr < ROWS; ++rr) {
        const int m = 16 * (4 * rr + wave) + r;
        xoff[rr] = ((m >> g.pw_log2) * g.xw + (m & (pw - 1))) * CP;
    }
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = 32 * s + 8 * kq;
        const int tap = k / CC < 9 ? k / CC : 8;
        toff[s] = ((tap / 3) * g.xw + tap % 3) * CP + k % CC;
    }
    const int woff = r * WS + 8 * kq;
    f32x4 acc[ROWS][NT];
#pragma unroll
    for (int rr = 0; rr < ROWS; ++rr)
#pragma unroll
        for (int tt = 0; tt < NT; ++tt) acc[rr][tt] = f32x4{0.f, 0.f, 0.f, 0.f};
    auto compute = [&]() {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            bf16x8 wf[NT];
#pragma unroll
            for (int tt = 0; tt < NT; ++tt) wf[tt] = *reinterpret_cast<const bf16x8 *>(&Ws[woff + 16 * WS * tt + 32 * s]);
#pragma unroll
            for (int rr = 0; rr < ROWS; ++rr) {
                const bf16x8 xf = *reinterpret_cast<const bf16x8 *>(&Xs[xoff[rr] + toff[s]]);
#pragma unroll
                for (int tt = 0; tt < NT; ++tt)
                    acc[rr][tt] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(wf[tt], xf, acc[rr][tt], 0, 0, 0);
            }
        }
    };

    load(0);
    stage();
    __syncthreads();
    for (int c0 = CC; c0 < g.Ci; c0 += CC) {
        load(c0);  // in flight while the current chunk is consumed
        // keep the loads ahead of the matrix instructions (the scheduler
        // would otherwise sink them next to their LDS writes)
        __builtin_amdgcn_sched_barrier(0);
        compute();
        __syncthreads();
        stage();
        __syncthreads();
    }
    compute();
    __syncthreads();  // the staging LDS becomes the output tile

    // accumulator element e of tile tt: channel co0 + 16 tt + 4 kq + e of the lane's pixel
    bf16 *const T = smem;
#pragma unroll
    for (int tt = 0; tt < NT; ++tt) {
        float bv[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) bv[e] = bias ? bias[co0 + 16 * tt + 4 * kq + e] : 0.f;
#pragma unroll
        for (int rr = 0; rr < ROWS; ++rr) {
            bf16x4 v;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                float f = acc[rr][tt][e] + bv[e];
                if (g.relu) f = fmaxf(f, 0.f);
                v[e] = (bf16)f;
            }
            *reinterpret_cast<bf16x4 *>(&T[(16 * (4 * rr + wave) + r) * TS + 16 * tt + 4 * kq]) = v;
        }
    }
    __syncthreads();
    constexpr int NG = NB / 8;  // 16-byte groups of a pixel's NB channels
    for (int u = t; u < 64 * ROWS * NG; u += 256) {
        const int m = u / NG, gq = u % NG;
        const int y = py0 + (m >> g.pw_log2), x = px0 + (m & (pw - 1));
        if (y < g.H && x < g.W)
            *reinterpret_cast<bf16x8 *>(out + (((long long)b * g.H + y) * g.W + x) * g.Co + co0 + 8 * gq) =
                *reinterpret_cast<const bf16x8 *>(&T[m * TS + 8 * gq]);
    }
    if (pooled) {
        const int hw = pw >> 1, Ho = g.H >> 1, Wo = g.W >> 1;
        for (int u = t; u < 16 * ROWS * NG; u += 256) {
            const int pm = u / NG, gq = u % NG;
            const int py = pm >> (g.pw_log2 - 1), pxl = pm & (hw - 1);
            const int Y = (py0 >> 1) + py, X = (px0 >> 1) + pxl;
            if (Y >= Ho || X >= Wo) continue;
            const int m00 = 2 * py * pw + 2 * pxl;
            const bf16x8 p00 = *reinterpret_cast<const bf16x8 *>(&T[m00 * TS + 8 * gq]);
            const bf16x8 p01 = *reinterpret_cast<const bf16x8 *>(&T[(m00 + 1) * TS + 8 * gq]);
            const bf16x8 p10 = *reinterpret_cast<const bf16x8 *>(&T[(m00 + pw) * TS + 8 * gq]);
            const bf16x8 p11 = *reinterpret_cast<const bf16x8 *>(&T[(m00 + pw + 1) * TS + 8 * gq]);
            bf16x8 o;
#pragma unroll
            for (int e = 0; e < 8; ++e)
                o[e] = (bf16)(0.25f * ((float)p00[e] + (float)p01[e] + (float)p10[e] + (float)p11[e]));
            *reinterpret_cast<bf16x8 *>(pooled + (((long long)b * Ho + Y) * Wo + X) * g.Co + co0 + 8 * gq) = o;
        }
    }
    if (head_out) {
        for (int m = t; m < 64 * ROWS; m += 256) {
            const int y = py0 + (m >> g.pw_log2), x = px0 + (m & (pw - 1));
            if (y >= g.H || x >= g.W) continue;
            for (int o = 0; o < g.head_o; ++o) {
                float sum = head_b[o];
#pragma unroll
                for (int c0 = 0; c0 < NB; c0 += 8) {
                    const bf16x8 xv = *reinterpret_cast<const bf16x8 *>(&T[m * TS + c0]);
#pragma unroll
                    for (int e = 0; e < 8; ++e) sum += (float)xv[e] * (float)head_w[o * NB + c0 + e];
                }
                head_out[(((long long)b * g.H + y) * g.W + x) * g.head_o + o] = sum;
            }
        }
    }
}

// The instantiated (ROWS, NB, CC): the staging registers (XU + WU units of
// 4 VGPRs) stay within 24 units and the LDS within 96 KB.
#define RLBM_CONV_VARIANTS(X)                                                                                   \
    X(4, 16, 16) X(4, 16, 32) X(4, 16, 64) X(4, 32, 16) X(4, 32, 32) X(4, 32, 64) X(4, 64, 16) X(4, 64, 32)     \
    X(2, 16, 16) X(2, 16, 32) X(2, 16, 64) X(2, 32, 16) X(2, 32, 32) X(2, 32, 64) X(2, 64, 16) X(2, 64, 32)     \
    X(1, 16, 16) X(1, 16, 32) X(1, 16, 64) X(1, 16, 128) X(1, 32, 16) X(1, 32, 32) X(1, 32, 64) X(1, 64, 16)    \
    X(1, 64, 32)

// wt[ci][8 - tap][co] = w[co][tap][ci]: the weights of the adjoint convolution.
__global__ void conv3x3_adjoint_weights_kernel(const bf16 *__restrict__ w, bf16 *__restrict__ wt, int Ci, int Co)
{
    const long long n = (long long)Co * 9 * Ci;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const int ci = (int)(q % Ci);
        const int tap = (int)((q / Ci) % 9);
        const int co = (int)(q / ((long long)Ci * 9));
        wt[((long long)ci * 9 + (8 - tap)) * Co + co] = w[q];
    }
}

// All layers' adjoint weights in one launch (one thread per source weight;
// the layer is found by a scan of the table's offsets).
__global__ void conv3x3_adjoint_all_kernel(const bf16 *__restrict__ w, bf16 *__restrict__ wt, const AdjointTable t)
{
    const long long n = t.toff[t.n];
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        int k = 0;
        while (k + 1 < t.n && q >= t.toff[k + 1]) ++k;
        const long long local = q - t.toff[k];
        const int Ci = t.ci[k], Co = t.co[k];
        const int ci = (int)(local % Ci);
        const int tap = (int)((local / Ci) % 9);
        const int co = (int)(local / ((long long)Ci * 9));
        wt[t.toff[k] + ((long long)ci * 9 + (8 - tap)) * Co + co] = w[t.woff[k] + local];
    }
}

// Weight gradient, one partial per chunk of image rows:
// part[chunk][co][tap][ci] = sum over the chunk's pixels p of
//   dpre[p][co] * in[p shifted by tap][ci]   (zero outside the image).
// A GEMM with M = co, N = ci, K = pixels for each of the 9 taps.  The sum is
// taken over the input pixel x' = x + dx - 1 of a row:
//   sum_x' dpre[y][x' + 1 - dx][co] * in[y + dy - 1][x'][ci]
// (the terms dropped or added at the image edges are zero on either side).
// A chunk is `per` consecutive rows of one image (chunk c: image c / cpi,
// rows from (c % cpi) * per), taken RB rows and one segment of SEG pixels
// at a time.  The matrix instructions want 8 consecutive pixels of one
// channel per lane, while NHWC keeps channels contiguous, so each segment
// is staged through LDS transposed: the CIB input channels of the RB + 2
// rows y-1 .. y+RB, Bs[row][ci][k], and for each of the RB rows the 16
// output channels in three copies shifted by the tap's dx, As[row][dx][co][k]
// (a 16-channel tile is cheaper to replicate than CIB channels), so that
// every operand is one aligned 16-byte LDS read.  A lane stages a pair of
// adjacent pixels: it loads both pixels' 8 channels (16-byte raw buffer
// loads; an offset past the buffer's end reads zero, which pads the image
// and the rows past the chunk) and writes each channel's pair as one 32-bit
// word, consecutive lanes taking consecutive pairs of one row.  The loads of
// the next step are in flight while the matrix instructions consume the
// current one.  CIB * SEG = 2048 (64 x 32, 32 x 64 or 16 x 128, by the input
// channel count): the four wavefronts take CIB / 16 channel tiles times
// SEG / 32 pixel quarters, each keeps the 9 taps' 16 x 16 accumulators over
// all its rows, and the quarters of a tile are added in order at the end.
// grid.x = chunks = B * cpi, grid.y = (Co / 16) * ceil(Ci / CIB).
template <int CIB, int RB>
__global__ __launch_bounds__(256) void conv3x3_wgrad_kernel(const bf16 *__restrict__ dpre,
                                                            const bf16 *__restrict__ in, float *__restrict__ part,
                                                            int B, int H, int W, int Ci, int Co, int cpi, int per)
{
    constexpr int SEG = 2048 / CIB, NCT = CIB / 16;
    constexpr int SP = SEG + 8;            // staged row of one channel: 16-byte aligned, padded
    constexpr int NP = SEG / 2;            // pixel pairs of a segment
    constexpr int G = CIB / 8;             // 16-byte groups of a pixel's CIB channels
    constexpr int XN = (RB + 2) * NP * G;  // input units: (row, group, pair)
    constexpr int XU = (XN + 255) / 256;
    constexpr int DN = RB * 2 * NP;        // output-gradient units: (row, group of 8 channels, pair)
    constexpr int DU = (DN + 255) / 256;
    // staging (As then Bs) and, at the end, the reduction of the four waves'
    // accumulators share one LDS buffer
    constexpr int kAs = RB * 3 * 16 * SP, kBs = (RB + 2) * CIB * SP;
    constexpr int kRed = 4 * 9 * 4 * 64 * (int)sizeof(float);
    constexpr int kBytes = (kAs + kBs) * (int)sizeof(bf16) > kRed ? (kAs + kBs) * (int)sizeof(bf16) : kRed;
    __shared__ __attribute__((aligned(16))) char smem[kBytes];
    bf16 *const As = reinterpret_cast<bf16 *>(smem);  // [RB][3][16][SP]
    bf16 *const Bs = As + kAs;                         // [RB + 2][CIB][SP]
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int ct = wave % NCT, kp = wave / NCT;
    const int cib = (Ci + CIB - 1) / CIB;
    const int og = blockIdx.y / cib, cb = blockIdx.y % cib;
    const int co0 = og * 16, ci0 = cb * CIB;
    const bool active = ci0 + 16 * ct < Ci;
    const int r = lane & 15, kq = lane >> 4;
    const int img = (int)blockIdx.x / cpi;
    const int y0 = ((int)blockIdx.x % cpi) * per, y1 = y0 + per < H ? y0 + per : H;
    const int nseg = (W + SEG - 1) / SEG;
    const int nit = y1 > y0 ? (y1 - y0 + RB - 1) / RB * nseg : 0;  // (row group, segment) steps
    constexpr unsigned kOut = 0x80000000u;
    const __amdgpu_buffer_rsrc_t xrs =
        __builtin_amdgcn_make_buffer_rsrc((void *)in, (short)0, B * H * W * Ci * 2, 0x00020000);
    const __amdgpu_buffer_rsrc_t drs =
        __builtin_amdgcn_make_buffer_rsrc((void *)dpre, (short)0, B * H * W * Co * 2, 0x00020000);
    // each unit's fixed part of its address, and whether it reads anything
    int xj[XU], xrow[XU], xc[XU], dj[DU], drow[DU], dc[DU];
    bool xv[XU], dvld[DU];
#pragma unroll
    for (int i = 0; i < XU; ++i) {
        const int u = t + 256 * i;
        const int j = u % NP, rest = u / NP, g = rest % G, rr = rest / G;
        xj[i] = 2 * j;
        xrow[i] = rr - 1;
        xc[i] = ci0 + 8 * g;
        xv[i] = (XN % 256 == 0 || u < XN) & (ci0 + 8 * g < Ci);
    }
#pragma unroll
    for (int i = 0; i < DU; ++i) {
        const int u = t + 256 * i;
        const int j = u % NP, rest = u / NP;
        dj[i] = 2 * j - 1;
        dc[i] = co0 + 8 * (rest % 2);
        drow[i] = rest / 2;
        dvld[i] = DN % 256 == 0 || u < DN;
    }
    bf16x8 xa[XU], xb[XU], dv[DU][4];
    auto load = [&](int it) {
        const int yg = y0 + (it / nseg) * RB, x0 = (it % nseg) * SEG;
#pragma unroll
        for (int i = 0; i < XU; ++i) {
            const int yy = yg + xrow[i], xx = x0 + xj[i];
            const bool ok = xv[i] & ((unsigned)yy < (unsigned)H);
            const unsigned o = (unsigned)((((img * H + yy) * W + xx) * Ci + xc[i]) * 2);
            const unsigned o0 = ok & (xx < W) ? o : kOut, o1 = ok & (xx + 1 < W) ? o + 2u * Ci : kOut;
            xa[i] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(xrs, (int)o0, 0, 0));
            xb[i] = __builtin_bit_cast(bf16x8, __builtin_amdgcn_raw_buffer_load_b128(xrs, (int)o1, 0, 0));
        }
#pragma unroll
        for (int i = 0; i < DU; ++i) {
            const int y = yg + drow[i], xs = x0 + dj[i];  // input pixels xs .. xs + 3 of a row of the chunk
            const unsigned o = (unsigned)((((img * H + y) * W + xs) * Co + dc[i]) * 2);
            const bool rok = dvld[i] & (y < y1);
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                const bool ok = rok & ((unsigned)(xs + q) < (unsigned)W);
                dv[i][q] = __builtin_bit_cast(
                    bf16x8, __builtin_amdgcn_raw_buffer_load_b128(drs, (int)(ok ? o + 2u * Co * q : kOut), 0, 0));
            }
        }
    };
    auto pack = [](bf16 lo, bf16 hi) {
        return (unsigned)__builtin_bit_cast(unsigned short, lo) | ((unsigned)__builtin_bit_cast(unsigned short, hi) << 16);
    };
    auto stage = [&]() {
#pragma unroll
        for (int i = 0; i < XU; ++i) {
            const int u = t + 256 * i;
            if (XN % 256 == 0 || u < XN) {
                const int j = u % NP, rest = u / NP, g = rest % G, rr = rest / G;
                bf16 *const p = Bs + (rr * CIB + 8 * g) * SP + 2 * j;
#pragma unroll
                for (int e = 0; e < 8; ++e) *reinterpret_cast<unsigned *>(p + e * SP) = pack(xa[i][e], xb[i][e]);
            }
        }
#pragma unroll
        for (int i = 0; i < DU; ++i) {
            const int u = t + 256 * i;
            if (DN % 256 == 0 || u < DN) {
                const int j = u % NP, rest = u / NP, g = rest % 2, rb = rest / 2;
                // As[rb][dx][co][k] = dpre[row rb][x0 + k + 1 - dx][co]: for k = 2j, 2j + 1
                // the pixels x0 + 2j + 1 - dx and x0 + 2j + 2 - dx, i.e. dv[2 - dx], dv[3 - dx]
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    bf16 *const p = As + ((rb * 3 + dx) * 16 + 8 * g) * SP + 2 * j;
#pragma unroll
                    for (int e = 0; e < 8; ++e)
                        *reinterpret_cast<unsigned *>(p + e * SP) = pack(dv[i][2 - dx][e], dv[i][3 - dx][e]);
                }
            }
        }
    };
    f32x4 acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    // no branch around the products: pixels past the image, rows past the
    // chunk and channels past Ci were staged as zeros, so an idle quarter,
    // row or tile adds zero (and an inactive tile's sums are not written)
    auto compute = [&]() {
#pragma unroll
        for (int rb = 0; rb < RB; ++rb) {
            bf16x8 a[3];
#pragma unroll
            for (int dx = 0; dx < 3; ++dx)
                a[dx] = *reinterpret_cast<const bf16x8 *>(&As[((rb * 3 + dx) * 16 + r) * SP + kp * 32 + kq * 8]);
#pragma unroll
            for (int dy = 0; dy < 3; ++dy) {
                const bf16x8 b =
                    *reinterpret_cast<const bf16x8 *>(&Bs[((rb + dy) * CIB + 16 * ct + r) * SP + kp * 32 + kq * 8]);
#pragma unroll
                for (int dx = 0; dx < 3; ++dx)
                    acc[dy * 3 + dx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[dx], b, acc[dy * 3 + dx], 0, 0, 0);
            }
        }
    };
    if (nit > 0) {
        load(0);
        stage();
        __syncthreads();
        for (int it = 0; it + 1 < nit; ++it) {
            load(it + 1);  // in flight while this step's products run
            __builtin_amdgcn_sched_barrier(0);
            compute();
            __syncthreads();
            stage();
            __syncthreads();
        }
        compute();
    }
    __syncthreads();  // the staging LDS becomes the reduction buffer
    // add the pixel quarters of each channel tile in order, through LDS
    float *red = reinterpret_cast<float *>(smem);  // 4 x 9 x 4 x 64 floats
#pragma unroll
    for (int tap = 0; tap < 9; ++tap)
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) red[((wave * 9 + tap) * 4 + s2) * 64 + lane] = acc[tap][s2];
    __syncthreads();
    if (!active || kp != 0) return;
    // C[i = co row][j = ci col] in lane j + 16*(i/4), element i%4
    float *o = part + (long long)blockIdx.x * Co * 9 * Ci;
    const int ci = ci0 + 16 * ct + (lane & 15);
#pragma unroll
    for (int tap = 0; tap < 9; ++tap) {
#pragma unroll
        for (int s2 = 0; s2 < 4; ++s2) {
            float v = 0.f;
#pragma unroll
            for (int q = 0; q < 4 / NCT; ++q) v += red[(((ct + q * NCT) * 9 + tap) * 4 + s2) * 64 + lane];
            const int co = co0 + 4 * (lane >> 4) + s2;
            o[((long long)co * 9 + tap) * Ci + ci] = v;
        }
    }
}

// g[q] += sum over chunks of part[chunk][q]: a block takes 16 entries q,
// its 16 thread groups the chunks c = group (mod 16), and the 16 group sums
// are added in group order (deterministic).
__global__ __launch_bounds__(256) void reduce_chunks_kernel(const float *__restrict__ part, float *__restrict__ g,
                                                            long long n, int chunks)
{
    const int qi = threadIdx.x & 15, grp = threadIdx.x >> 4;
    const long long q = (long long)blockIdx.x * 16 + qi;
    float s = 0.f;
    if (q < n) {
        // four chunks' loads in flight per pass, added in chunk order
        int c = grp;
        for (; c + 48 < chunks; c += 64) {
            const float v0 = part[(long long)c * n + q], v1 = part[(long long)(c + 16) * n + q];
            const float v2 = part[(long long)(c + 32) * n + q], v3 = part[(long long)(c + 48) * n + q];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; c < chunks; c += 16) s += part[(long long)c * n + q];
    }
    __shared__ float red[16][16];
    red[grp][qi] = s;
    __syncthreads();
    if (grp == 0 && q < n) {
        float t = 0.f;
        for (int k = 0; k < 16; ++k) t += red[k][qi];
        g[q] += t;
    }
}

// The deferred reductions of a backward pass in one launch: block b belongs
// to the job whose block range holds it and sums 64 of that job's outputs
// over all chunks; wave w takes the chunks c = w (mod 4), four loads in
// flight, each a 256-byte row segment of one chunk, and the four wave sums
// are added in wave order (deterministic).
__global__ __launch_bounds__(256) void reduce_jobs_kernel(const ReduceJobs J)
{
    const long long b = blockIdx.x;
    int j = 0;
    while (j + 1 < J.n && b >= J.block_start[j + 1]) ++j;
    const float *__restrict__ part = J.part[j];
    const long long n = J.len[j];
    const int chunks = J.chunks[j];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const long long q = (b - J.block_start[j]) * 64 + lane;
    float s = 0.f;
    if (q < n) {
        int c = w;
        for (; c + 12 < chunks; c += 16) {
            const float v0 = part[(long long)c * n + q], v1 = part[(long long)(c + 4) * n + q];
            const float v2 = part[(long long)(c + 8) * n + q], v3 = part[(long long)(c + 12) * n + q];
            s += v0;
            s += v1;
            s += v2;
            s += v3;
        }
        for (; c < chunks; c += 4) s += part[(long long)c * n + q];
    }
    __shared__ float red[4][64];
    red[w][lane] = s;
    __syncthreads();
    if (w == 0 && q < n) J.g[j][q] += ((red[0][lane] + red[1][lane]) + red[2][lane]) + red[3][lane];
}

// Per-channel sums in two passes (deterministic: fixed partition, fixed
// order), optionally fused with the ReLU gradient.  Pass 1: block b sums
// the pixels of its chunk; thread t takes the eight channels 8 (t % G) ..
// of pixels t / G, t / G + 256 / G, ... (G = C / 8 groups, one 16-byte
// load each), applying d *= (out > 0) first when `out` is given; the block
// adds up its 256 / G rows in a fixed tree and writes part[b][c].  Needs
// C % 8 == 0 and G | 256.
__global__ __launch_bounds__(256) void channel_sum_part_kernel(bf16 *__restrict__ d, const bf16 *__restrict__ out,
                                                               float *__restrict__ part, long long npix, int C,
                                                               long long chunk)
{
    const int t = threadIdx.x;
    const int G = C / 8;
    const int g = t % G, r = t / G, rows = 256 / G;
    const long long p0 = (long long)blockIdx.x * chunk;
    const long long p1 = p0 + chunk < npix ? p0 + chunk : npix;
    float acc[8];
#pragma unroll
    for (int e = 0; e < 8; ++e) acc[e] = 0.f;
    // four pixel rows per pass, all loads issued before any is used; the
    // additions keep the pixel order p, p + rows, p + 2 rows, ...
    constexpr int U = 4;
    for (long long p = p0 + r; p < p1; p += U * rows) {
        bf16x8 v[U], o[U];
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const long long pk = p + (long long)k * rows;
            if (pk < p1) {
                v[k] = *reinterpret_cast<const bf16x8 *>(d + pk * C + 8 * g);
                if (out) o[k] = *reinterpret_cast<const bf16x8 *>(out + pk * C + 8 * g);
            }
        }
#pragma unroll
        for (int k = 0; k < U; ++k) {
            const long long pk = p + (long long)k * rows;
            if (pk >= p1) break;
            if (out) {
#pragma unroll
                for (int e = 0; e < 8; ++e)
                    if (!((float)o[k][e] > 0.f)) v[k][e] = (bf16)0.f;
                *reinterpret_cast<bf16x8 *>(d + pk * C + 8 * g) = v[k];
            }
#pragma unroll
            for (int e = 0; e < 8; ++e) acc[e] += (float)v[k][e];
        }
    }
    __shared__ float red[256][9];
#pragma unroll
    for (int e = 0; e < 8; ++e) red[t][e] = acc[e];
    __syncthreads();
    for (int k = 128; k >= G; k >>= 1) {
        if (t < k) {
#pragma unroll
            for (int e = 0; e < 8; ++e) red[t][e] += red[t + k][e];
        }
        __syncthreads();
    }
    if (t < G) {
#pragma unroll
        for (int e = 0; e < 8; ++e) part[(long long)blockIdx.x * C + 8 * t + e] = red[t][e];
    }
}

// Fallback for channel counts that do not divide 256: one block per channel.
__global__ __launch_bounds__(256) void channel_sum_kernel(const bf16 *__restrict__ d, float *__restrict__ gb,
                                                          long long npix, int C)
{
    const int c = blockIdx.x;
    float s = 0.f;
    for (long long p = threadIdx.x; p < npix; p += blockDim.x) s += (float)d[p * C + c];
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) gb[c] += red[0];
}

// Pass 2: g[c] += sum over the nb blocks of part[b][c]; one block per
// entry c, a fixed-shape tree over the blocks (deterministic).
__global__ __launch_bounds__(256) void sum_parts_kernel(const float *__restrict__ part, float *__restrict__ g, int nb,
                                                        int n)
{
    const int c = blockIdx.x;
    float s = 0.f;
    for (int b = threadIdx.x; b < nb; b += 256) s += part[(long long)b * n + c];
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) g[c] += red[0];
}

// d *= (out > 0): gradient through the ReLU of a layer with output `out`.
__global__ void relu_backward_kernel(bf16 *__restrict__ d, const bf16 *__restrict__ out, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        if (!((float)out[q] > 0.f)) d[q] = (bf16)0.f;
}

// ---------------------------------------------------------------- resampling

// The resampling kernels move 8 channels (16 bytes) per thread: every
// channel count and channel offset here is a multiple of 8 (the launchers
// check), so a group never straddles two tensors.  Each element's arithmetic
// is the same as channel by channel.

// out (B, H/2, W/2, C) = mean of 2x2 blocks of in (B, H, W, C)
__global__ void pool_fwd_kernel(const bf16 *__restrict__ in, bf16 *__restrict__ out, int B, int H, int W, int C)
{
    const int Ho = H / 2, Wo = W / 2, C8 = C / 8;
    const long long n = (long long)B * Ho * Wo * C8;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const int c = 8 * (int)(q % C8);
        long long t = q / C8;
        const int x = (int)(t % Wo);
        t /= Wo;
        const int y = (int)(t % Ho);
        const int b = (int)(t / Ho);
        const long long base = (((long long)b * H + 2 * y) * W + 2 * x) * C + c;
        const bf16x8 p00 = *reinterpret_cast<const bf16x8 *>(in + base);
        const bf16x8 p01 = *reinterpret_cast<const bf16x8 *>(in + base + C);
        const bf16x8 p10 = *reinterpret_cast<const bf16x8 *>(in + base + (long long)W * C);
        const bf16x8 p11 = *reinterpret_cast<const bf16x8 *>(in + base + (long long)W * C + C);
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e)
            o[e] = (bf16)(0.25f * ((float)p00[e] + (float)p01[e] + (float)p10[e] + (float)p11[e]));
        *reinterpret_cast<bf16x8 *>(out + 8 * q) = o;
    }
}

// dx (B, H, W, C) = dy / 4 broadcast (+ skip, a (B, H, W, Cs) tensor's channels [off, off + C))
__global__ void pool_bwd_kernel(const bf16 *__restrict__ dy, const bf16 *__restrict__ skip, int skip_c, int skip_off,
                                bf16 *__restrict__ dx, int B, int H, int W, int C)
{
    const int C8 = C / 8;
    const long long n = (long long)B * H * W * C8;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const int c = 8 * (int)(q % C8);
        const long long pix = q / C8;
        const int x = (int)(pix % W);
        const long long t = pix / W;
        const int y = (int)(t % H);
        const int b = (int)(t / H);
        const bf16x8 g = *reinterpret_cast<const bf16x8 *>(dy + (((long long)b * (H / 2) + y / 2) * (W / 2) + x / 2) * C + c);
        bf16x8 k;
        if (skip) k = *reinterpret_cast<const bf16x8 *>(skip + pix * skip_c + skip_off + c);
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) {
            float v = 0.25f * (float)g[e];
            if (skip) v += (float)k[e];
            o[e] = (bf16)v;
        }
        *reinterpret_cast<bf16x8 *>(dx + 8 * q) = o;
    }
}

// cat (B, H, W, Cu + Cs): channels [0, Cu) = nearest x2 upsample of u (B, H/2, W/2, Cu),
// channels [Cu, Cu + Cs) = s (B, H, W, Cs)
__global__ void up_concat_kernel(const bf16 *__restrict__ u, const bf16 *__restrict__ s, bf16 *__restrict__ cat, int B,
                                 int H, int W, int Cu, int Cs)
{
    const int C8 = (Cu + Cs) / 8, Cu8 = Cu / 8;
    const long long n = (long long)B * H * W * C8;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const int c8 = (int)(q % C8);
        const long long pix = q / C8;
        bf16x8 v;
        if (c8 < Cu8) {
            const int x = (int)(pix % W);
            const long long t = pix / W;
            const int y = (int)(t % H);
            const int b = (int)(t / H);
            v = *reinterpret_cast<const bf16x8 *>(u + (((long long)b * (H / 2) + y / 2) * (W / 2) + x / 2) * Cu + 8 * c8);
        } else {
            v = *reinterpret_cast<const bf16x8 *>(s + pix * Cs + 8 * (c8 - Cu8));
        }
        *reinterpret_cast<bf16x8 *>(cat + 8 * q) = v;
    }
}

// du (B, H/2, W/2, Cu) = sum over each 2x2 block of dcat's channels [0, Cu)
__global__ void up_bwd_kernel(const bf16 *__restrict__ dcat, bf16 *__restrict__ du, int B, int H, int W, int Cu,
                              int C)
{
    const int Ho = H / 2, Wo = W / 2, Cu8 = Cu / 8;
    const long long n = (long long)B * Ho * Wo * Cu8;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const int c = 8 * (int)(q % Cu8);
        long long t = q / Cu8;
        const int x = (int)(t % Wo);
        t /= Wo;
        const int y = (int)(t % Ho);
        const int b = (int)(t / Ho);
        const long long base = (((long long)b * H + 2 * y) * W + 2 * x) * C + c;
        const bf16x8 p00 = *reinterpret_cast<const bf16x8 *>(dcat + base);
        const bf16x8 p01 = *reinterpret_cast<const bf16x8 *>(dcat + base + C);
        const bf16x8 p10 = *reinterpret_cast<const bf16x8 *>(dcat + base + (long long)W * C);
        const bf16x8 p11 = *reinterpret_cast<const bf16x8 *>(dcat + base + (long long)W * C + C);
        bf16x8 o;
#pragma unroll
        for (int e = 0; e < 8; ++e) o[e] = (bf16)((float)p00[e] + (float)p01[e] + (float)p10[e] + (float)p11[e]);
        *reinterpret_cast<bf16x8 *>(du + 8 * q) = o;
    }
}

// ---------------------------------------------------------------- head, loss, optimiser

// y[p][o] = b[o] + sum_c x[p][c] * w[o][c]   (1x1 convolution, FP32 output)
// One thread per pixel, its channels read 8 at a time (16 bytes; C is a
// multiple of 8), each output summed over the channels in ascending order.
__global__ void head_fwd_kernel(const bf16 *__restrict__ x, const bf16 *__restrict__ w, const float *__restrict__ b,
                                float *__restrict__ y, long long npix, int C, int O)
{
    for (long long p = blockIdx.x * (long long)blockDim.x + threadIdx.x; p < npix; p += (long long)gridDim.x * blockDim.x) {
        const bf16 *xp = x + p * C;
        for (int o = 0; o < O; ++o) {
            float s = b[o];
            for (int c0 = 0; c0 < C; c0 += 8) {
                const bf16x8 xv = *reinterpret_cast<const bf16x8 *>(xp + c0);
#pragma unroll
                for (int e = 0; e < 8; ++e) s += (float)xv[e] * (float)w[o * C + c0 + e];
            }
            y[p * O + o] = s;
        }
    }
}

// dx[p][c] = sum_o dy[p][o] * w[o][c]  (BF16 output)
__global__ void head_bwd_data_kernel(const float *__restrict__ dy, const bf16 *__restrict__ w, bf16 *__restrict__ dx,
                                     long long npix, int C, int O)
{
    const long long n = npix * C;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const int c = (int)(q % C);
        const long long p = q / C;
        float s = 0.f;
        for (int o = 0; o < O; ++o) s += dy[p * O + o] * (float)w[o * C + c];
        dx[q] = (bf16)s;
    }
}

// Head parameter gradient for other shapes: one block per output entry
// (o, c) of W (c < C) or of the bias (c == C).
__global__ __launch_bounds__(256) void head_wgrad_kernel(const float *__restrict__ dy, const bf16 *__restrict__ x,
                                                         float *__restrict__ gw, float *__restrict__ gb,
                                                         long long npix, int C, int O)
{
    const int o = blockIdx.x / (C + 1), c = blockIdx.x % (C + 1);
    float s = 0.f;
    for (long long p = threadIdx.x; p < npix; p += blockDim.x) s += dy[p * O + o] * (c < C ? (float)x[p * C + c] : 1.f);
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        if (c < C)
            gw[o * C + c] += red[0];
        else
            gb[o] += red[0];
    }
}

// Head parameter gradient, pass 1: block b covers a chunk of pixels, each
// thread its pixels t, t + 256, ...; every thread keeps the O * (C + 1)
// sums dy[p][o] x[p][c] (c < C) and dy[p][o] (the bias, c = C), the block
// adds them up (wavefront shuffles, then across the four wavefronts) and
// writes part[b][o * (C + 1) + c].  Pass 2 is sum_parts_kernel.
template <int C, int O>
__global__ __launch_bounds__(256) void head_wgrad_part_kernel(const float *__restrict__ dy, const bf16 *__restrict__ x,
                                                              float *__restrict__ part, long long npix,
                                                              long long chunk)
{
    constexpr int K = O * (C + 1);
    float acc[K];
#pragma unroll
    for (int k = 0; k < K; ++k) acc[k] = 0.f;
    const long long p0 = (long long)blockIdx.x * chunk;
    const long long p1 = p0 + chunk < npix ? p0 + chunk : npix;
    for (long long p = p0 + threadIdx.x; p < p1; p += 256) {
        float g[O], xv[C];
#pragma unroll
        for (int o = 0; o < O; ++o) g[o] = dy[p * O + o];
#pragma unroll
        for (int c = 0; c < C; ++c) xv[c] = (float)x[p * C + c];
#pragma unroll
        for (int o = 0; o < O; ++o) {
#pragma unroll
            for (int c = 0; c < C; ++c) acc[o * (C + 1) + c] += g[o] * xv[c];
            acc[o * (C + 1) + C] += g[o];
        }
    }
    __shared__ float red[4][K];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int k = 0; k < K; ++k) {
        float v = acc[k];
        for (int m = 32; m > 0; m >>= 1) v += __shfl_xor(v, m);
        if (lane == 0) red[wave][k] = v;
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += 256)
        part[(long long)blockIdx.x * K + k] = red[0][k] + red[1][k] + red[2][k] + red[3][k];
}

// Head parameter gradient, pass 2: gw[o][c] and gb[o] += the block sums of
// part (rows of O * (C + 1) entries); one block per entry, a fixed tree.
__global__ __launch_bounds__(256) void head_grad_scatter_kernel(const float *__restrict__ part, float *__restrict__ gw,
                                                                float *__restrict__ gb, int nb, int C, int O)
{
    const int k = blockIdx.x;
    const int K = O * (C + 1);
    float s = 0.f;
    for (int b = threadIdx.x; b < nb; b += 256) s += part[(long long)b * K + k];
    __shared__ float red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int m = 128; m > 0; m >>= 1) {
        if ((int)threadIdx.x < m) red[threadIdx.x] += red[threadIdx.x + m];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        const int o = k / (C + 1), c = k % (C + 1);
        if (c < C)
            gw[o * C + c] += red[0];
        else
            gb[o] += red[0];
    }
}

// Mean squared error: per-block partial sums of (y - t)^2 and dy = 2 (y - t) / n.
__global__ __launch_bounds__(256) void mse_kernel(const float *__restrict__ y, const float *__restrict__ t,
                                                  float *__restrict__ dy, double *__restrict__ part, long long n)
{
    double s = 0.0;
    const float scale = 2.0f / (float)n;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const float d = y[q] - t[q];
        s += (double)d * d;
        if (dy) dy[q] = scale * d;
    }
    __shared__ double red[256];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k > 0; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// Adam with bias correction; keeps the FP32 master parameters and refreshes
// their BF16 copies (conv weights) in the same pass.
__global__ void adam_kernel(float *__restrict__ theta, const float *__restrict__ g, float *__restrict__ m,
                            float *__restrict__ v, bf16 *__restrict__ theta_bf, long long n, float lr, float b1,
                            float b2, float eps, float c1, float c2)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x) {
        const float gq = g[q];
        const float mq = b1 * m[q] + (1.f - b1) * gq;
        const float vq = b2 * v[q] + (1.f - b2) * gq * gq;
        m[q] = mq;
        v[q] = vq;
        const float th = theta[q] - lr * (mq / c1) / (sqrtf(vq / c2) + eps);
        theta[q] = th;
        theta_bf[q] = (bf16)th;
    }
}

__global__ void to_bf16_kernel(const float *__restrict__ a, bf16 *__restrict__ b, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        b[q] = (bf16)a[q];
}

// Four values per thread (16-byte loads, 8-byte stores); n4 = n / 4, both
// arrays 16-byte aligned (the launcher checks and takes the scalar kernel
// otherwise and for the tail).
__global__ void to_bf16_x4_kernel(const float4 *__restrict__ a, bf16 *__restrict__ b, long long n4)
{
    typedef __attribute__((__vector_size__(4 * sizeof(__bf16)))) __bf16 bf16x4_t;
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n4; q += (long long)gridDim.x * blockDim.x) {
        const float4 v = a[q];
        bf16x4_t o;
        o[0] = (bf16)v.x;
        o[1] = (bf16)v.y;
        o[2] = (bf16)v.z;
        o[3] = (bf16)v.w;
        *reinterpret_cast<bf16x4_t *>(b + 4 * q) = o;
    }
}

__global__ void to_f32_kernel(const bf16 *__restrict__ a, float *__restrict__ b, long long n)
{
    for (long long q = blockIdx.x * (long long)blockDim.x + threadIdx.x; q < n; q += (long long)gridDim.x * blockDim.x)
        b[q] = (float)a[q];
}

inline unsigned grid_for(long long n, int block = 256)
{
    long long g = (n + block - 1) / block;
    if (g > 65536) g = 65536;
    if (g < 1) g = 1;
    return (unsigned)g;
}

}  // namespace

hipError_t conv3x3_forward_ex(const ConvInputs &x, const void *w, const float *bias, void *out, int B, int H, int W,
                              int Ci, int Co, bool relu, hipStream_t s)
{
    if (Ci % 16 || Co % 16 || B < 1 || H < 1 || W < 1 || !x.in) return hipErrorInvalidValue;
    // one image's input is addressed with 32-bit byte offsets (buffer loads)
    if ((long long)H * W * Ci * 2 >= (1LL << 31)) return hipErrorInvalidValue;
    ConvGeom g;
    g.H = H;
    g.W = W;
    g.Ci = Ci;
    g.Co = Co;
    g.pw_log2 = W > 32 ? 6 : W > 16 ? 5 : 4;
    g.xw = (1 << g.pw_log2) + 2;
    g.xw_magic = (unsigned)((1ull << 32) / (unsigned)g.xw + 1);  // exact below 2^16 for xw <= 66
    g.patches_x = (W + (1 << g.pw_log2) - 1) >> g.pw_log2;
    g.relu = relu ? 1 : 0;
    g.cu = Ci;
    g.head_o = 0;
    // The largest patch x channel tile that still gives 512 blocks (two per
    // compute unit), else the one with the most blocks.
    static const int kTiles[][2] = {{4, 64}, {4, 32}, {2, 64}, {4, 16}, {2, 32}, {1, 64}, {2, 16}, {1, 32}, {1, 16}};
    int rows = 0, nb = 0;
    long long best = -1;
    for (const auto &c : kTiles) {
        if (Co % c[1]) continue;
        const int pr = (64 * c[0]) >> g.pw_log2;
        const long long blocks = (long long)B * ((H + pr - 1) / pr) * g.patches_x * (Co / c[1]);
        if (blocks > best) {
            best = blocks;
            rows = c[0];
            nb = c[1];
        }
        if (blocks >= 512) {
            rows = c[0];
            nb = c[1];
            break;
        }
    }
    const int pr = (64 * rows) >> g.pw_log2;
    g.patches_y = (H + pr - 1) / pr;
    const long long gx = (long long)B * g.patches_y * g.patches_x;
    if (gx > 0x7fffffffLL) return hipErrorInvalidValue;
    const dim3 grid((unsigned)gx, (unsigned)(Co / nb));

    // A concatenation is read in place: both parts are multiples of 16
    // channels, so a chunk width divides both and a chunk lies in one part.
    const bf16 *in = static_cast<const bf16 *>(x.in);
    const bf16 *skip = nullptr;
    const bool cat = x.skip != nullptr;
    if (cat) {
        if (x.cu < 16 || x.cu >= Ci || x.cu % 16 || H % 2 || W % 2) return hipErrorInvalidValue;
        skip = static_cast<const bf16 *>(x.skip);
        g.cu = x.cu;
    }
    int cc = 0;
    for (int c = 128; c >= 16 && !cc; c /= 2)
        if (Ci % c == 0 && (!cat || (x.cu % c == 0 && (Ci - x.cu) % c == 0))) cc = c;
    // the pooled copy and the head come from the block's output tile when
    // the patch holds whole 2x2 blocks / all output channels
    const bool pool_fused = x.pooled && pr % 2 == 0;
    const bool head_fused = x.head_out && nb == Co;
    bf16 *o = static_cast<bf16 *>(out);
    bf16 *pooled = pool_fused ? static_cast<bf16 *>(x.pooled) : nullptr;
    const bf16 *hw = head_fused ? static_cast<const bf16 *>(x.head_w) : nullptr;
    float *hout = head_fused ? x.head_out : nullptr;
    if (head_fused) g.head_o = x.head_o;
    const bf16 *wt = static_cast<const bf16 *>(w);
    bool launched = false;
    // the widest instantiated chunk that fits; every tile has a CC = 16 variant
    for (int c = cc; c >= 16 && !launched; c /= 2) {
        if (Ci % c || (cat && (g.cu % c || (Ci - g.cu) % c))) continue;
#define RLBM_CONV_LAUNCH(R, N, C)                                                                                   \
    if (!launched && rows == R && nb == N && c == C) {                                                             \
        if (cat)                                                                                                   \
            hipLaunchKernelGGL((conv3x3_fwd_kernel<R, N, C, true>), grid, dim3(256), 0, s, in, skip, wt, bias, o,  \
                               pooled, hw, x.head_b, hout, g);                                                     \
        else                                                                                                       \
            hipLaunchKernelGGL((conv3x3_fwd_kernel<R, N, C, false>), grid, dim3(256), 0, s, in, skip, wt, bias, o, \
                               pooled, hw, x.head_b, hout, g);                                                     \
        launched = true;                                                                                           \
    }
        RLBM_CONV_VARIANTS(RLBM_CONV_LAUNCH)
#undef RLBM_CONV_LAUNCH
    }
    if (!launched) return hipErrorInvalidValue;
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (x.pooled && !pool_fused) e = pool_forward(out, x.pooled, B, H, W, Co, s);
    if (e == hipSuccess && x.head_out && !head_fused)
        e = head_forward(out, x.head_w, x.head_b, x.head_out, (long long)B * H * W, Co, x.head_o, s);
    return e;
}

hipError_t conv3x3_forward(const void *in, const void *w, const float *bias, void *out, int B, int H, int W, int Ci,
                           int Co, bool relu, hipStream_t s)
{
    ConvInputs x;
    x.in = in;
    return conv3x3_forward_ex(x, w, bias, out, B, H, W, Ci, Co, relu, s);
}

hipError_t conv3x3_adjoint_weights_all(const void *w, void *wt, const AdjointTable &t, hipStream_t s)
{
    if (t.n < 1 || t.n > kMaxAdjoint) return hipErrorInvalidValue;
    hipLaunchKernelGGL(conv3x3_adjoint_all_kernel, dim3(grid_for(t.toff[t.n])), dim3(256), 0, s,
                       static_cast<const bf16 *>(w), static_cast<bf16 *>(wt), t);
    return hipGetLastError();
}

hipError_t conv3x3_adjoint_weights(const void *w, void *wt, int Ci, int Co, hipStream_t s)
{
    hipLaunchKernelGGL(conv3x3_adjoint_weights_kernel, dim3(grid_for((long long)Co * 9 * Ci)), dim3(256), 0, s,
                       static_cast<const bf16 *>(w), static_cast<bf16 *>(wt), Ci, Co);
    return hipGetLastError();
}

namespace {
// input channels staged per block of the weight gradient
int wgrad_cib(int Ci) { return Ci == 16 ? 16 : Ci == 32 ? 32 : 64; }
}  // namespace

namespace {
// Chunks of the weight gradient: about 512 blocks in all (chunks x channel
// tiles), each chunk `per` whole rows of one image, cpi chunks per image.
void wgrad_split(int B, int H, int Ci, int Co, int &cpi, int &per)
{
    const int cib = wgrad_cib(Ci);
    const long long tiles = (long long)(Co / 16) * ((Ci + cib - 1) / cib);
    const long long target = (512 + tiles - 1) / tiles;
    long long c = (target + B - 1) / B;
    if (c > H) c = H;
    if (c < 1) c = 1;
    per = (int)((H + c - 1) / c);
    cpi = (H + per - 1) / per;
}
}  // namespace

int conv3x3_wgrad_chunks(int B, int H, int W, int Ci, int Co)
{
    int cpi = 0, per = 0;
    wgrad_split(B, H, Ci, Co, cpi, per);
    (void)W;
    return B * cpi;
}

int conv3x3_backward_weight_part(const void *dpre, const void *in, float *part, int B, int H, int W, int Ci, int Co,
                                 hipStream_t s)
{
    if (Ci % 16 || Co % 16 || B < 1 || H < 1 || W < 1) return -1;
    // both tensors are addressed with 32-bit byte offsets (buffer loads)
    if ((long long)B * H * W * (Ci > Co ? Ci : Co) * 2 >= (1LL << 31)) return -1;
    int cpi = 0, per = 0;
    wgrad_split(B, H, Ci, Co, cpi, per);
    const int chunks = B * cpi;
    const int cib = wgrad_cib(Ci);
    const dim3 grid(chunks, (Co / 16) * ((Ci + cib - 1) / cib));
    const bf16 *d = static_cast<const bf16 *>(dpre), *x = static_cast<const bf16 *>(in);
    // rows per step: up to four, no more than a chunk holds
    const int rb = per >= 4 ? 4 : per >= 2 ? 2 : 1;
#define RLBM_WGRAD(C, R)                                                                                      \
    if (cib == C && rb == R)                                                                                  \
        hipLaunchKernelGGL((conv3x3_wgrad_kernel<C, R>), grid, dim3(256), 0, s, d, x, part, B, H, W, Ci, Co, cpi, per);
    RLBM_WGRAD(16, 1) RLBM_WGRAD(16, 2) RLBM_WGRAD(16, 4) RLBM_WGRAD(32, 1) RLBM_WGRAD(32, 2) RLBM_WGRAD(32, 4)
    RLBM_WGRAD(64, 1) RLBM_WGRAD(64, 2) RLBM_WGRAD(64, 4)
#undef RLBM_WGRAD
    return hipGetLastError() == hipSuccess ? chunks : -1;
}

hipError_t conv3x3_backward_weight(const void *dpre, const void *in, float *part, float *gw, int B, int H, int W,
                                   int Ci, int Co, hipStream_t s)
{
    const int chunks = conv3x3_backward_weight_part(dpre, in, part, B, H, W, Ci, Co, s);
    if (chunks < 0) return hipErrorInvalidValue;
    const long long n = (long long)Co * 9 * Ci;
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((n + 15) / 16)), dim3(256), 0, s, part, gw, n, chunks);
    return hipGetLastError();
}

bool add_reduce_job(ReduceJobs &j, const float *part, float *g, long long len, int chunks)
{
    if (j.n >= kMaxReduceJobs || len < 1 || chunks < 1) return false;
    j.part[j.n] = part;
    j.g[j.n] = g;
    j.len[j.n] = len;
    j.chunks[j.n] = chunks;
    j.block_start[j.n + 1] = j.block_start[j.n] + (len + 63) / 64;
    ++j.n;
    return true;
}

hipError_t reduce_partials(const ReduceJobs &j, hipStream_t s)
{
    if (j.n == 0) return hipSuccess;
    const long long blocks = j.block_start[j.n];
    if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
    hipLaunchKernelGGL(reduce_jobs_kernel, dim3((unsigned)blocks), dim3(256), 0, s, j);
    return hipGetLastError();
}

int channel_sum_blocks(long long npix)
{
    const long long b = (npix + 255) / 256;  // at least 256 pixels per block
    return (int)(b < kSumBlocks ? (b < 1 ? 1 : b) : kSumBlocks);
}

namespace {
bool fast_sum_shape(int C) { return C >= 8 && C % 8 == 0 && C <= 2048 && 256 % (C / 8) == 0; }

hipError_t sum_launch(bf16 *d, const bf16 *out, float *part, float *gb, long long npix, int C, hipStream_t s)
{
    const int nb = channel_sum_blocks(npix);
    const long long chunk = (npix + nb - 1) / nb;
    hipLaunchKernelGGL(channel_sum_part_kernel, dim3(nb), dim3(256), 0, s, d, out, part, npix, C, chunk);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(sum_parts_kernel, dim3(C), dim3(256), 0, s, part, gb, nb, C);
    return hipGetLastError();
}
}  // namespace

hipError_t channel_sum(const void *d, float *part, float *gb, long long npix, int C, hipStream_t s)
{
    if (C < 1 || npix < 1) return hipErrorInvalidValue;
    if (!fast_sum_shape(C)) {
        hipLaunchKernelGGL(channel_sum_kernel, dim3(C), dim3(256), 0, s, static_cast<const bf16 *>(d), gb, npix, C);
        return hipGetLastError();
    }
    // no ReLU: the kernel only reads d
    return sum_launch(static_cast<bf16 *>(const_cast<void *>(d)), nullptr, part, gb, npix, C, s);
}

hipError_t relu_backward_bias_part(void *d, const void *out, float *part, float *gb, long long npix, int C, int *rows,
                                   hipStream_t s)
{
    *rows = 0;
    if (C < 1 || npix < 1) return hipErrorInvalidValue;
    if (!fast_sum_shape(C)) return relu_backward_bias(d, out, part, gb, npix, C, s);
    const int nb = channel_sum_blocks(npix);
    const long long chunk = (npix + nb - 1) / nb;
    hipLaunchKernelGGL(channel_sum_part_kernel, dim3(nb), dim3(256), 0, s, static_cast<bf16 *>(d),
                       static_cast<const bf16 *>(out), part, npix, C, chunk);
    *rows = nb;
    return hipGetLastError();
}

hipError_t relu_backward_bias(void *d, const void *out, float *part, float *gb, long long npix, int C, hipStream_t s)
{
    if (C < 1 || npix < 1) return hipErrorInvalidValue;
    if (!fast_sum_shape(C)) {
        hipError_t e = relu_backward(d, out, npix * C, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(channel_sum_kernel, dim3(C), dim3(256), 0, s, static_cast<const bf16 *>(d), gb, npix, C);
        return hipGetLastError();
    }
    return sum_launch(static_cast<bf16 *>(d), static_cast<const bf16 *>(out), part, gb, npix, C, s);
}

hipError_t relu_backward(void *d, const void *out, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(relu_backward_kernel, dim3(grid_for(n)), dim3(256), 0, s, static_cast<bf16 *>(d),
                       static_cast<const bf16 *>(out), n);
    return hipGetLastError();
}

hipError_t pool_forward(const void *in, void *out, int B, int H, int W, int C, hipStream_t s)
{
    if (C % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pool_fwd_kernel, dim3(grid_for((long long)B * H * W * C / 32)), dim3(256), 0, s,
                       static_cast<const bf16 *>(in), static_cast<bf16 *>(out), B, H, W, C);
    return hipGetLastError();
}

hipError_t pool_backward(const void *dy, const void *skip, int skip_c, int skip_off, void *dx, int B, int H, int W,
                         int C, hipStream_t s)
{
    if (C % 8 || (skip && (skip_c % 8 || skip_off % 8))) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pool_bwd_kernel, dim3(grid_for((long long)B * H * W * C / 8)), dim3(256), 0, s,
                       static_cast<const bf16 *>(dy), static_cast<const bf16 *>(skip), skip_c, skip_off,
                       static_cast<bf16 *>(dx), B, H, W, C);
    return hipGetLastError();
}

hipError_t up_concat(const void *u, const void *skip, void *cat, int B, int H, int W, int Cu, int Cs, hipStream_t s)
{
    if (Cu % 8 || Cs % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(up_concat_kernel, dim3(grid_for((long long)B * H * W * (Cu + Cs) / 8)), dim3(256), 0, s,
                       static_cast<const bf16 *>(u), static_cast<const bf16 *>(skip), static_cast<bf16 *>(cat), B, H,
                       W, Cu, Cs);
    return hipGetLastError();
}

hipError_t up_backward(const void *dcat, void *du, int B, int H, int W, int Cu, int C, hipStream_t s)
{
    if (Cu % 8 || C % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(up_bwd_kernel, dim3(grid_for((long long)B * H * W * Cu / 32)), dim3(256), 0, s,
                       static_cast<const bf16 *>(dcat), static_cast<bf16 *>(du), B, H, W, Cu, C);
    return hipGetLastError();
}

hipError_t head_forward(const void *x, const void *w, const float *b, float *y, long long npix, int C, int O,
                        hipStream_t s)
{
    if (C % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(head_fwd_kernel, dim3(grid_for(npix)), dim3(256), 0, s, static_cast<const bf16 *>(x),
                       static_cast<const bf16 *>(w), b, y, npix, C, O);
    return hipGetLastError();
}

hipError_t head_backward(const float *dy, const void *x, const void *w, void *dx, float *part, float *gw, float *gb,
                         long long npix, int C, int O, hipStream_t s)
{
    if (C < 1 || O < 1 || npix < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(head_bwd_data_kernel, dim3(grid_for(npix * C)), dim3(256), 0, s, dy,
                       static_cast<const bf16 *>(w), static_cast<bf16 *>(dx), npix, C, O);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (C != 16 || O != 3) {
        hipLaunchKernelGGL(head_wgrad_kernel, dim3(O * (C + 1)), dim3(256), 0, s, dy, static_cast<const bf16 *>(x), gw,
                           gb, npix, C, O);
        return hipGetLastError();
    }
    // at most 256 blocks (at least eight pixels per thread at 256 x 256 x 8):
    // each block ends in a reduction of its 51 sums, which one pixel per
    // thread would leave as the kernel's main cost
    const int nb = channel_sum_blocks(npix) < 256 ? channel_sum_blocks(npix) : 256;
    const long long chunk = (npix + nb - 1) / nb;
    hipLaunchKernelGGL((head_wgrad_part_kernel<16, 3>), dim3(nb), dim3(256), 0, s, dy, static_cast<const bf16 *>(x),
                       part, npix, chunk);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(head_grad_scatter_kernel, dim3(O * (C + 1)), dim3(256), 0, s, part, gw, gb, nb, C, O);
    return hipGetLastError();
}

hipError_t mse(const float *y, const float *t, float *dy, double *part, int nblocks, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(mse_kernel, dim3(nblocks), dim3(256), 0, s, y, t, dy, part, n);
    return hipGetLastError();
}

hipError_t adam(float *theta, const float *g, float *m, float *v, void *theta_bf, long long n, float lr, float b1,
                float b2, float eps, float c1, float c2, hipStream_t s)
{
    hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n)), dim3(256), 0, s, theta, g, m, v, static_cast<bf16 *>(theta_bf),
                       n, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t to_bf16(const float *a, void *b, long long n, hipStream_t s)
{
    if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(b)) % 16 == 0 && n >= 4) {
        const long long n4 = n / 4;
        hipLaunchKernelGGL(to_bf16_x4_kernel, dim3(grid_for(n4)), dim3(256), 0, s, reinterpret_cast<const float4 *>(a),
                           static_cast<bf16 *>(b), n4);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess || n4 * 4 == n) return e;
        hipLaunchKernelGGL(to_bf16_kernel, dim3(1), dim3(256), 0, s, a + 4 * n4, static_cast<bf16 *>(b) + 4 * n4,
                           n - 4 * n4);
        return hipGetLastError();
    }
    hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n)), dim3(256), 0, s, a, static_cast<bf16 *>(b), n);
    return hipGetLastError();
}

hipError_t to_f32(const void *a, float *b, long long n, hipStream_t s)
{
    hipLaunchKernelGGL(to_f32_kernel, dim3(grid_for(n)), dim3(256), 0, s, static_cast<const bf16 *>(a), b, n);
    return hipGetLastError();
}

}  // namespace rlbm
