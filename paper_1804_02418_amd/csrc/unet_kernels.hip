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

template <int KSTEP>
struct Mfma;
template <>
struct Mfma<32> {
    typedef bf16x8 vec;
    __device__ static f32x4 run(vec a, vec b, f32x4 c) { return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0); }
};
template <>
struct Mfma<16> {
    typedef bf16x4 vec;
    __device__ static f32x4 run(vec a, vec b, f32x4 c)
    {
        typedef __attribute__((__vector_size__(4 * sizeof(short)))) short s4;
        return __builtin_amdgcn_mfma_f32_16x16x16bf16_1k(__builtin_bit_cast(s4, a), __builtin_bit_cast(s4, b), c, 0, 0,
                                                         0);
    }
};

// ---------------------------------------------------------------- conv 3x3

// grid.x = B * ceil(H / ROWS) * ceil(W / 64), grid.y = Co / 16; 4
// wavefronts per block, wavefront w covers pixels x0 + 16 w ... + 15 of
// ROWS consecutive output rows.  The block stages the ROWS + 2 input rows it
// needs (66 pixels: the segment and one on each side, zero outside the
// image) and its 16 output channels' weights through LDS, CC input channels
// at a time (16, 32 or 64: the LDS a block holds follows the layer's width,
// so narrow layers keep more blocks resident), so that every input value is
// fetched once per block instead of once per tap and wavefront, and each
// staged row serves up to three output rows.
template <int KSTEP, bool RELU, int ROWS, int CC>
__global__ __launch_bounds__(256) void conv3x3_fwd_kernel(const bf16 *__restrict__ in, const bf16 *__restrict__ w,
                                                          const float *__restrict__ bias, bf16 *__restrict__ out,
                                                          int H, int W, int Ci, int Co)
{
    typedef typename Mfma<KSTEP>::vec vec;
    constexpr int KPL = KSTEP / 4;  // channels per lane per K step
    constexpr int CP = CC + 8;      // CC channels per chunk, padded row (fewer bank conflicts)
    __shared__ __attribute__((aligned(16))) bf16 Xs[ROWS + 2][66][CP];
    __shared__ __attribute__((aligned(16))) bf16 Ws[16][9][CP];
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int tiles_w = (W + 63) / 64;
    const int groups_h = (H + ROWS - 1) / ROWS;
    int q = blockIdx.x;
    const int xt = q % tiles_w;
    q /= tiles_w;
    const int y0 = (q % groups_h) * ROWS;
    const int b = q / groups_h;
    const int xs = xt * 64, x0 = xs + wave * 16;
    const int co0 = blockIdx.y * 16;
    const int r = lane & 15;   // A row (pixel) and B column (channel)
    const int kq = lane >> 4;  // which group of KPL channels
    f32x4 acc[ROWS];
#pragma unroll
    for (int rr = 0; rr < ROWS; ++rr) acc[rr] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16 z = (bf16)0.f;
    for (int c0 = 0; c0 < Ci; c0 += CC) {
        const int cc = Ci - c0 < CC ? Ci - c0 : CC;  // a multiple of 16
        const int groups = cc / 8;
        for (int unit = t; unit < (ROWS + 2) * 66 * groups; unit += 256) {
            const int g = unit % groups, rest = unit / groups;
            const int u = rest % 66, rr = rest / 66;
            const int yy = y0 + rr - 1, xx = xs + u - 1;
            bf16x8 v;
            if ((unsigned)yy < (unsigned)H && (unsigned)xx < (unsigned)W)
                v = *reinterpret_cast<const bf16x8 *>(in + (((long long)b * H + yy) * W + xx) * Ci + c0 + 8 * g);
            else
                for (int e = 0; e < 8; ++e) v[e] = z;
            *reinterpret_cast<bf16x8 *>(&Xs[rr][u][8 * g]) = v;
        }
        for (int unit = t; unit < 16 * 9 * groups; unit += 256) {
            const int g = unit % groups, rest = unit / groups;
            const int tap = rest % 9, co = rest / 9;
            *reinterpret_cast<bf16x8 *>(&Ws[co][tap][8 * g]) =
                *reinterpret_cast<const bf16x8 *>(w + ((long long)(co0 + co) * 9 + tap) * Ci + c0 + 8 * g);
        }
        __syncthreads();
        if (x0 < W) {
#pragma unroll
            for (int tap = 0; tap < 9; ++tap) {
                const int dy = tap / 3, dx = tap % 3;
                for (int k0 = 0; k0 < cc; k0 += KSTEP) {
                    const vec bv = *reinterpret_cast<const vec *>(&Ws[r][tap][k0 + kq * KPL]);
#pragma unroll
                    for (int rr = 0; rr < ROWS; ++rr) {
                        const vec a = *reinterpret_cast<const vec *>(&Xs[rr + dy][wave * 16 + r + dx][k0 + kq * KPL]);
                        acc[rr] = Mfma<KSTEP>::run(a, bv, acc[rr]);
                    }
                }
            }
        }
        __syncthreads();
    }
    if (x0 >= W) return;
    const int j = lane & 15;
    const float bj = bias ? bias[co0 + j] : 0.f;
#pragma unroll
    for (int rr = 0; rr < ROWS; ++rr) {
        const int y = y0 + rr;
        if (y >= H) break;
#pragma unroll
        for (int s = 0; s < 4; ++s) {
            const int px = x0 + 4 * (lane >> 4) + s;
            if (px < W) {
                float v = acc[rr][s] + bj;
                if (RELU) v = fmaxf(v, 0.f);
                out[(((long long)b * H + y) * W + px) * Co + co0 + j] = (bf16)v;
            }
        }
    }
}

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
// The matrix instructions want 8 consecutive pixels of one channel per
// lane, while NHWC keeps channels contiguous, so each row segment of SEG
// input pixels is staged through LDS transposed: the CIB input channels of
// the rows y-1, y, y+1 once, Bs[row][ci][k], and the 16 output channels in
// three copies shifted by the tap's dx, As[dx][co][k] (a 16-channel tile is
// cheaper to replicate than CIB channels), so that every operand is one
// aligned 16-byte LDS read.  CIB * SEG = 2048 (64 x 32, 32 x 64 or 16 x 128,
// by the input channel count): the four wavefronts take CIB / 16 channel
// tiles times SEG / 32 pixel quarters, each keeps the 9 taps' 16 x 16
// accumulators, and the quarters of a tile are added in order at the end.
// grid.x = chunks (whole rows each), grid.y = (Co / 16) * ceil(Ci / CIB).
template <int CIB>
__global__ __launch_bounds__(256) void conv3x3_wgrad_kernel(const bf16 *__restrict__ dpre,
                                                            const bf16 *__restrict__ in, float *__restrict__ part,
                                                            int B, int H, int W, int Ci, int Co, int rows_per_chunk)
{
    constexpr int SEG = 2048 / CIB, NCT = CIB / 16;
    // staging (As then Bs) and, at the end, the reduction of the four waves'
    // accumulators share one LDS buffer
    constexpr int kAs = 3 * 16 * SEG, kBs = 3 * CIB * SEG;
    constexpr int kRed = 4 * 9 * 4 * 64 * (int)sizeof(float);
    constexpr int kBytes = (kAs + kBs) * (int)sizeof(bf16) > kRed ? (kAs + kBs) * (int)sizeof(bf16) : kRed;
    __shared__ __attribute__((aligned(16))) char smem[kBytes];
    bf16 (*As)[16][SEG] = reinterpret_cast<bf16 (*)[16][SEG]>(smem);
    bf16 (*Bs)[CIB][SEG] = reinterpret_cast<bf16 (*)[CIB][SEG]>(smem + kAs * sizeof(bf16));
    const int t = threadIdx.x, wave = t >> 6, lane = t & 63;
    const int ct = wave % NCT, kp = wave / NCT;
    const int cib = (Ci + CIB - 1) / CIB;
    const int og = blockIdx.y / cib, cb = blockIdx.y % cib;
    const int co0 = og * 16, ci0 = cb * CIB;
    const bool active = ci0 + 16 * ct < Ci;
    const int r = lane & 15, kq = lane >> 4;
    const long long row0 = (long long)blockIdx.x * rows_per_chunk;
    const long long rows_end = row0 + rows_per_chunk < (long long)B * H ? row0 + rows_per_chunk : (long long)B * H;
    f32x4 acc[9];
#pragma unroll
    for (int q = 0; q < 9; ++q) acc[q] = f32x4{0.f, 0.f, 0.f, 0.f};
    const bf16 z = (bf16)0.f;
    for (long long gr = row0; gr < rows_end; ++gr) {
        const int y = (int)(gr % H);
        const long long img = gr / H;
        for (int x0 = 0; x0 < W; x0 += SEG) {
            const int seg = W - x0 < SEG ? W - x0 : SEG;
            // ---- stage dpre: pixels x0-1 .. x0+SEG, 16 channels, two per
            // unit; pixel x0 + u serves shift dx at k = u - 1 + dx
            for (int unit = t; unit < (SEG + 2) * 8; unit += 256) {
                const int u = unit / 8 - 1, cp = (unit % 8) * 2;
                const int xx = x0 + u;
                bf16 v0 = z, v1 = z;
                if ((unsigned)xx < (unsigned)W) {
                    const bf16 *q = dpre + ((img * H + y) * W + xx) * Co + co0 + cp;
                    v0 = q[0];
                    v1 = q[1];
                }
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) {
                    const int k = u - 1 + dx;
                    if (k >= 0 && k < SEG) {
                        As[dx][cp][k] = v0;
                        As[dx][cp + 1][k] = v1;
                    }
                }
            }
            // ---- stage in: rows y-1..y+1, pixels x0 .. x0+SEG-1, CIB channels
            // in groups of 8
            for (int unit = t; unit < 3 * SEG * (CIB / 8); unit += 256) {
                const int g = unit % (CIB / 8), rest = unit / (CIB / 8);
                const int k = rest % SEG, rr = rest / SEG;
                const int yy = y + rr - 1, xx = x0 + k, c = ci0 + 8 * g;
                bf16x8 v;
                if ((unsigned)yy < (unsigned)H && xx < W && c < Ci)
                    v = *reinterpret_cast<const bf16x8 *>(in + ((img * H + yy) * W + xx) * Ci + c);
                else
                    for (int e = 0; e < 8; ++e) v[e] = z;
#pragma unroll
                for (int e = 0; e < 8; ++e) Bs[rr][8 * g + e][k] = v[e];
            }
            __syncthreads();
            if (active && kp * 32 < seg) {
                bf16x8 a[3];
#pragma unroll
                for (int dx = 0; dx < 3; ++dx) a[dx] = *reinterpret_cast<const bf16x8 *>(&As[dx][r][kp * 32 + kq * 8]);
#pragma unroll
                for (int dy = 0; dy < 3; ++dy) {
                    const bf16x8 b = *reinterpret_cast<const bf16x8 *>(&Bs[dy][16 * ct + r][kp * 32 + kq * 8]);
#pragma unroll
                    for (int dx = 0; dx < 3; ++dx)
                        acc[dy * 3 + dx] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a[dx], b, acc[dy * 3 + dx], 0, 0, 0);
                }
            }
            __syncthreads();
        }
    }
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

hipError_t conv3x3_forward(const void *in, const void *w, const float *bias, void *out, int B, int H, int W, int Ci,
                           int Co, bool relu, hipStream_t s)
{
    if (Ci % 16 || Co % 16 || B < 1 || H < 1 || W < 1) return hipErrorInvalidValue;
    const bf16 *i = static_cast<const bf16 *>(in), *wt = static_cast<const bf16 *>(w);
    bf16 *o = static_cast<bf16 *>(out);
    // four output rows per block on images of 16 rows or more (each staged
    // row then serves up to three output rows; measured faster than one row
    // per block down to the 16 x 16 level of a 256 x 256 network), one on
    // smaller images; channel chunks of the layer's width up to 64
    const bool four = H >= 16;
    const dim3 grid((unsigned)(B * (four ? (H + 3) / 4 : H) * ((W + 63) / 64)), (unsigned)(Co / 16));
#define RLBM_CONV_FWD(K, R, CC)                                                                                  \
    do {                                                                                                        \
        if (relu)                                                                                               \
            hipLaunchKernelGGL((conv3x3_fwd_kernel<K, true, R, CC>), grid, dim3(256), 0, s, i, wt, bias, o, H, W, Ci, Co); \
        else                                                                                                    \
            hipLaunchKernelGGL((conv3x3_fwd_kernel<K, false, R, CC>), grid, dim3(256), 0, s, i, wt, bias, o, H, W, Ci, Co); \
    } while (0)
    if (Ci == 16) {
        if (four)
            RLBM_CONV_FWD(16, 4, 16);
        else
            RLBM_CONV_FWD(16, 1, 16);
    } else if (Ci == 32) {
        if (four)
            RLBM_CONV_FWD(32, 4, 32);
        else
            RLBM_CONV_FWD(32, 1, 32);
    } else if (Ci % 32 == 0) {
        if (four)
            RLBM_CONV_FWD(32, 4, 64);
        else
            RLBM_CONV_FWD(32, 1, 64);
    } else {
        if (four)
            RLBM_CONV_FWD(16, 4, 64);
        else
            RLBM_CONV_FWD(16, 1, 64);
    }
#undef RLBM_CONV_FWD
    return hipGetLastError();
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

int conv3x3_wgrad_chunks(int B, int H, int W, int Ci, int Co)
{
    // about 1024 blocks in all (chunks x channel tiles), whole rows each
    const long long rows = (long long)B * H;
    const int cib = wgrad_cib(Ci);
    const long long tiles = (long long)(Co / 16) * ((Ci + cib - 1) / cib);
    long long chunks = (1024 + tiles - 1) / tiles;
    if (chunks > rows) chunks = rows;
    if (chunks < 1) chunks = 1;
    (void)W;
    return (int)chunks;
}

hipError_t conv3x3_backward_weight(const void *dpre, const void *in, float *part, float *gw, int B, int H, int W,
                                   int Ci, int Co, hipStream_t s)
{
    if (Ci % 16 || Co % 16 || B < 1 || H < 1 || W < 1) return hipErrorInvalidValue;
    const int chunks = conv3x3_wgrad_chunks(B, H, W, Ci, Co);
    const int per = (int)(((long long)B * H + chunks - 1) / chunks);
    const int cib = wgrad_cib(Ci);
    const dim3 grid(chunks, (Co / 16) * ((Ci + cib - 1) / cib));
    const bf16 *d = static_cast<const bf16 *>(dpre), *x = static_cast<const bf16 *>(in);
    if (cib == 16)
        hipLaunchKernelGGL(conv3x3_wgrad_kernel<16>, grid, dim3(256), 0, s, d, x, part, B, H, W, Ci, Co, per);
    else if (cib == 32)
        hipLaunchKernelGGL(conv3x3_wgrad_kernel<32>, grid, dim3(256), 0, s, d, x, part, B, H, W, Ci, Co, per);
    else
        hipLaunchKernelGGL(conv3x3_wgrad_kernel<64>, grid, dim3(256), 0, s, d, x, part, B, H, W, Ci, Co, per);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const long long n = (long long)Co * 9 * Ci;
    hipLaunchKernelGGL(reduce_chunks_kernel, dim3((unsigned)((n + 15) / 16)), dim3(256), 0, s, part, gw, n, chunks);
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
    const int nb = channel_sum_blocks(npix);
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
