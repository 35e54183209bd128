// Bandwidth probes (measurement helper; see include/rlbm_probe.h): read,
// copy and the step's 48-plane pull pattern with trivial arithmetic, timed
// with HIP events.  Every index is bounded: the read and copy kernels test
// each element index against the element count, and the pull kernel
// touches only sites with x, y in [5, n - 5), whose sources lie inside the
// 48-plane array.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <string>

#include "../../include/rlbm_probe.h"
#include "rlbm_math.h"

namespace rlbm {
rlbm_status set_error(rlbm_status st, const char *msg);
}

using namespace rlbm;

namespace {

// Read and copy: each block moves 1024 consecutive 16-byte elements, each
// thread four of them 256 apart (coalesced), all loads issued before any
// store so that four requests per thread are in flight.
constexpr int kPerThread = 4;

__global__ __launch_bounds__(256) void probe_read(const float4 *__restrict__ a, float *__restrict__ sink, size_t n)
{
    const size_t base = (size_t)blockIdx.x * (256 * kPerThread) + threadIdx.x;
    float4 v[kPerThread];
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) {
        const size_t i = base + (size_t)u * 256;
        v[u] = i < n ? a[i] : make_float4(0.f, 0.f, 0.f, 0.f);
    }
    float s = 0.f;
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) s += v[u].x + v[u].y + v[u].z + v[u].w;
    // a store the compiler cannot drop, which (the array being zero) never happens
    if (s == -1.0f) sink[0] = s;
}

template <bool NT>
__global__ __launch_bounds__(256) void probe_copy(const float4 *__restrict__ a, float4 *__restrict__ b, size_t n)
{
    const size_t base = (size_t)blockIdx.x * (256 * kPerThread) + threadIdx.x;
    float4 v[kPerThread];
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) {
        const size_t i = base + (size_t)u * 256;
        if (i < n) v[u] = a[i];
    }
#pragma unroll
    for (int u = 0; u < kPerThread; ++u) {
        const size_t i = base + (size_t)u * 256;
        if (i >= n) continue;
        if constexpr (NT) {
            __builtin_nontemporal_store(v[u].x, &b[i].x);
            __builtin_nontemporal_store(v[u].y, &b[i].y);
            __builtin_nontemporal_store(v[u].z, &b[i].z);
            __builtin_nontemporal_store(v[u].w, &b[i].w);
        } else {
            b[i] = v[u];
        }
    }
}

// One interior site per thread: the 48 hop-shifted loads of a pull, their
// sum as the only arithmetic, and 48 aligned stores.
template <class T, bool NT>
__global__ __launch_bounds__(256) void probe_pull48(const T *__restrict__ src, T *__restrict__ dst, int nx, int ny,
                                                   long long P)
{
    const int x = blockIdx.x * 256 + threadIdx.x;
    const int y = kReach + blockIdx.y;
    if (x < kReach || x >= nx - kReach || y >= ny - kReach) return;
    const long long site = (long long)y * nx + x;
    float h[kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int d = i / kShells;
        h[i] = (float)src[(long long)i * P + site - ((long long)kCy[d] * nx + kCx[d])];
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < kQ; ++i) s += h[i];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const T v = (T)(0.5f * h[i] + 1e-9f * s);
        if constexpr (NT)
            __builtin_nontemporal_store(v, &dst[(long long)i * P + site]);
        else
            dst[(long long)i * P + site] = v;
    }
}

// Two adjacent interior sites per thread (x even): each of the 48 planes is
// read as one two-element vector from the hop-shifted pair address (aligned
// to the element only, for odd hops) and written as one aligned vector.
template <class T>
struct Pair;
template <>
struct Pair<_Float16> {
    typedef unsigned int V __attribute__((aligned(2)));
    __device__ static float lo(V v) { return (float)__builtin_bit_cast(_Float16, (unsigned short)(v & 0xffffu)); }
    __device__ static float hi(V v) { return (float)__builtin_bit_cast(_Float16, (unsigned short)(v >> 16)); }
    __device__ static V make(float a, float b)
    {
        return (unsigned)__builtin_bit_cast(unsigned short, (_Float16)a) |
               ((unsigned)__builtin_bit_cast(unsigned short, (_Float16)b) << 16);
    }
};
typedef float pair_f32 __attribute__((ext_vector_type(2)));
typedef double pair_f64 __attribute__((ext_vector_type(2)));
template <>
struct Pair<float> {
    typedef pair_f32 V __attribute__((aligned(4)));
    __device__ static float lo(V v) { return v.x; }
    __device__ static float hi(V v) { return v.y; }
    __device__ static V make(float a, float b) { return V{a, b}; }
};
template <>
struct Pair<double> {
    typedef pair_f64 V __attribute__((aligned(8)));
    __device__ static float lo(V v) { return (float)v.x; }
    __device__ static float hi(V v) { return (float)v.y; }
    __device__ static V make(float a, float b) { return V{(double)a, (double)b}; }
};

template <class T, bool NT>
__global__ __launch_bounds__(256) void probe_pull48_pair(const T *__restrict__ src, T *__restrict__ dst, int nx,
                                                         int ny, long long P)
{
    typedef typename Pair<T>::V V;
    const int x = 2 * (blockIdx.x * 256 + threadIdx.x);
    const int y = kReach + blockIdx.y;
    if (x < kReach + 1 || x + 1 >= nx - kReach || y >= ny - kReach) return;
    const long long site = (long long)y * nx + x;
    float h[2 * kQ];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int d = i / kShells;
        const V v = *reinterpret_cast<const V *>(src + ((long long)i * P + site - ((long long)kCy[d] * nx + kCx[d])));
        h[2 * i] = Pair<T>::lo(v);
        h[2 * i + 1] = Pair<T>::hi(v);
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < 2 * kQ; ++i) s += h[i];
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const V v = Pair<T>::make(0.5f * h[2 * i] + 1e-9f * s, 0.5f * h[2 * i + 1] + 1e-9f * s);
        V *q = reinterpret_cast<V *>(dst + ((long long)i * P + site));
        if constexpr (NT)
            __builtin_nontemporal_store(v, q);
        else
            *q = v;
    }
}

// Direction-tuple layouts: the shells of one direction hop alike, so W of
// them (W = 4: all, W = 2: two) can sit together at each site: 48 / W
// arrays of nx*ny tuples of W elements.  One interior site per thread:
// 48 / W hop-shifted tuple loads, trivial arithmetic, 48 / W aligned tuple
// stores.
template <class T, int W, int TX, bool NT>
__global__ __launch_bounds__(256) void probe_pull_tuple(const T *__restrict__ src, T *__restrict__ dst, int nx,
                                                        int ny, long long P)
{
    typedef T V __attribute__((ext_vector_type(W)));
    // blocks of TX x (256 / TX) sites, as the step's tiles
    const int x = blockIdx.x * TX + (int)(threadIdx.x % TX);
    const int y = kReach + blockIdx.y * (256 / TX) + (int)(threadIdx.x / TX);
    if (x < kReach || x >= nx - kReach || y >= ny - kReach) return;
    const long long site = (long long)y * nx + x;
    const V *sv = reinterpret_cast<const V *>(src);
    V *dv = reinterpret_cast<V *>(dst);
    float h[kQ];
#pragma unroll
    for (int g = 0; g < kQ / W; ++g) {
        const int d = g * W / kShells;
        const V v = sv[(long long)g * P + site - ((long long)kCy[d] * nx + kCx[d])];
#pragma unroll
        for (int j = 0; j < W; ++j) h[W * g + j] = (float)v[j];
    }
    float s = 0.f;
#pragma unroll
    for (int i = 0; i < kQ; ++i) s += h[i];
#pragma unroll
    for (int g = 0; g < kQ / W; ++g) {
        V v;
#pragma unroll
        for (int j = 0; j < W; ++j) v[j] = (T)(0.5f * h[W * g + j] + 1e-9f * s);
        if constexpr (NT)
            __builtin_nontemporal_store(v, &dv[(long long)g * P + site]);
        else
            dv[(long long)g * P + site] = v;
    }
}

template <class T, int W, int TX = 256>
hipError_t launch_pull_tuple(const void *a, void *b, int nx, int ny, int nt, hipStream_t s)
{
    const dim3 grid((unsigned)((nx + TX - 1) / TX), (unsigned)((ny - 2 * kReach + 256 / TX - 1) / (256 / TX)));
    const long long P = (long long)nx * ny;
    if (nt)
        hipLaunchKernelGGL((probe_pull_tuple<T, W, TX, true>), grid, dim3(256), 0, s, static_cast<const T *>(a),
                           static_cast<T *>(b), nx, ny, P);
    else
        hipLaunchKernelGGL((probe_pull_tuple<T, W, TX, false>), grid, dim3(256), 0, s, static_cast<const T *>(a),
                           static_cast<T *>(b), nx, ny, P);
    return hipGetLastError();
}

template <class T>
hipError_t launch_pull_pair(const void *a, void *b, int nx, int ny, int nt, hipStream_t s)
{
    const dim3 grid((unsigned)((nx / 2 + 255) / 256), (unsigned)(ny - 2 * kReach));
    const long long P = (long long)nx * ny;
    if (nt)
        hipLaunchKernelGGL((probe_pull48_pair<T, true>), grid, dim3(256), 0, s, static_cast<const T *>(a),
                           static_cast<T *>(b), nx, ny, P);
    else
        hipLaunchKernelGGL((probe_pull48_pair<T, false>), grid, dim3(256), 0, s, static_cast<const T *>(a),
                           static_cast<T *>(b), nx, ny, P);
    return hipGetLastError();
}

template <class T>
hipError_t launch_pull(const void *a, void *b, int nx, int ny, int nt, hipStream_t s)
{
    const dim3 grid((unsigned)((nx + 255) / 256), (unsigned)(ny - 2 * kReach));
    const long long P = (long long)nx * ny;
    if (nt)
        hipLaunchKernelGGL((probe_pull48<T, true>), grid, dim3(256), 0, s, static_cast<const T *>(a),
                           static_cast<T *>(b), nx, ny, P);
    else
        hipLaunchKernelGGL((probe_pull48<T, false>), grid, dim3(256), 0, s, static_cast<const T *>(a),
                           static_cast<T *>(b), nx, ny, P);
    return hipGetLastError();
}

rlbm_status probe_fail(rlbm_status st, const char *what, hipError_t e)
{
    const std::string m = std::string("rlbm_bandwidth_probe: ") + what + ": " + hipGetErrorString(e);
    return set_error(e == hipErrorOutOfMemory ? RLBM_ENOMEM : st, m.c_str());
}

}  // namespace

extern "C" rlbm_status rlbm_bandwidth_probe(int pattern, int elem_bytes, int nx, int ny, int nontemporal, int reps,
                                            void *hip_stream, double *gbs, double *us)
{
    if (pattern < RLBM_PROBE_READ || pattern > RLBM_PROBE_PULL12_TUPLE_T64 ||
        (elem_bytes != 2 && elem_bytes != 4 && elem_bytes != 8) || nx <= 2 * kReach + 2 || ny <= 2 * kReach ||
        ny - 2 * kReach > 65535 || reps < 1 || (pattern == RLBM_PROBE_PULL48_PAIR && nx % 2))
        return set_error(RLBM_EINVAL, "rlbm_bandwidth_probe: invalid pattern, element size, size or repetitions");
    const size_t bytes = (size_t)kQ * (size_t)nx * (size_t)ny * (size_t)elem_bytes;
    if (bytes > (1ull << 34)) return set_error(RLBM_EINVAL, "rlbm_bandwidth_probe: array beyond 2^34 bytes");
    // 48 x elem_bytes is a multiple of 16, so the array is whole float4s
    const size_t n4 = bytes / 16;
    hipStream_t s = static_cast<hipStream_t>(hip_stream);
    void *a = nullptr, *b = nullptr;
    float *sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMalloc(&a, bytes);
    if (e == hipSuccess && pattern != RLBM_PROBE_READ) e = hipMalloc(&b, bytes);
    if (e == hipSuccess) e = hipMalloc((void **)&sink, sizeof(float));
    if (e == hipSuccess) e = hipMemsetAsync(a, 0, bytes, s);
    if (e == hipSuccess && b) e = hipMemsetAsync(b, 0, bytes, s);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    const unsigned grid = (unsigned)((n4 + 256 * kPerThread - 1) / (256 * kPerThread));
    auto one = [&](int k) -> hipError_t {
        if (pattern == RLBM_PROBE_READ) {
            hipLaunchKernelGGL(probe_read, dim3(grid), dim3(256), 0, s, static_cast<const float4 *>(a), sink, n4);
            return hipGetLastError();
        }
        if (pattern == RLBM_PROBE_COPY) {
            if (nontemporal)
                hipLaunchKernelGGL((probe_copy<true>), dim3(grid), dim3(256), 0, s, static_cast<const float4 *>(a),
                                   static_cast<float4 *>(b), n4);
            else
                hipLaunchKernelGGL((probe_copy<false>), dim3(grid), dim3(256), 0, s, static_cast<const float4 *>(a),
                                   static_cast<float4 *>(b), n4);
            return hipGetLastError();
        }
        const void *from = (k & 1) ? b : a;
        void *to = (k & 1) ? a : b;
        if (pattern == RLBM_PROBE_PULL12_TUPLE)
            return elem_bytes == 2 ? launch_pull_tuple<_Float16, 4>(from, to, nx, ny, nontemporal, s)
                   : elem_bytes == 4 ? launch_pull_tuple<float, 4>(from, to, nx, ny, nontemporal, s)
                                     : launch_pull_tuple<double, 4>(from, to, nx, ny, nontemporal, s);
        if (pattern == RLBM_PROBE_PULL24_TUPLE)
            return elem_bytes == 2 ? launch_pull_tuple<_Float16, 2>(from, to, nx, ny, nontemporal, s)
                   : elem_bytes == 4 ? launch_pull_tuple<float, 2>(from, to, nx, ny, nontemporal, s)
                                     : launch_pull_tuple<double, 2>(from, to, nx, ny, nontemporal, s);
        if (pattern >= RLBM_PROBE_PULL48_T64) {
            const int w = pattern == RLBM_PROBE_PULL48_T64 ? 1 : pattern == RLBM_PROBE_PULL24_TUPLE_T64 ? 2 : 4;
            if (elem_bytes == 2)
                return w == 1 ? launch_pull_tuple<_Float16, 1, 64>(from, to, nx, ny, nontemporal, s)
                       : w == 2 ? launch_pull_tuple<_Float16, 2, 64>(from, to, nx, ny, nontemporal, s)
                                : launch_pull_tuple<_Float16, 4, 64>(from, to, nx, ny, nontemporal, s);
            if (elem_bytes == 4)
                return w == 1 ? launch_pull_tuple<float, 1, 64>(from, to, nx, ny, nontemporal, s)
                       : w == 2 ? launch_pull_tuple<float, 2, 64>(from, to, nx, ny, nontemporal, s)
                                : launch_pull_tuple<float, 4, 64>(from, to, nx, ny, nontemporal, s);
            return w == 1 ? launch_pull_tuple<double, 1, 64>(from, to, nx, ny, nontemporal, s)
                   : w == 2 ? launch_pull_tuple<double, 2, 64>(from, to, nx, ny, nontemporal, s)
                            : launch_pull_tuple<double, 4, 64>(from, to, nx, ny, nontemporal, s);
        }
        if (pattern == RLBM_PROBE_PULL48_PAIR)
            return elem_bytes == 2 ? launch_pull_pair<_Float16>(from, to, nx, ny, nontemporal, s)
                   : elem_bytes == 4 ? launch_pull_pair<float>(from, to, nx, ny, nontemporal, s)
                                     : launch_pull_pair<double>(from, to, nx, ny, nontemporal, s);
        return elem_bytes == 2 ? launch_pull<_Float16>(from, to, nx, ny, nontemporal, s)
               : elem_bytes == 4 ? launch_pull<float>(from, to, nx, ny, nontemporal, s)
                                 : launch_pull<double>(from, to, nx, ny, nontemporal, s);
    };
    for (int k = 0; k < 3 && e == hipSuccess; ++k) e = one(k);
    if (e == hipSuccess) e = hipEventRecord(e0, s);
    for (int k = 0; k < reps && e == hipSuccess; ++k) e = one(k + 1);
    if (e == hipSuccess) e = hipEventRecord(e1, s);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    float ms = 0.f;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
    const hipError_t ee = e;
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    (void)hipFree(a);
    (void)hipFree(b);
    (void)hipFree(sink);
    if (ee != hipSuccess) return probe_fail(RLBM_EDEVICE, "device", ee);
    const double t = (double)ms / reps * 1e-3;
    // the pair pattern covers the pairs (x, x + 1), x even, inside [6, nx - 5)
    const double interior = (double)(pattern == RLBM_PROBE_PULL48_PAIR ? 2 * ((nx - kReach - 1 - (kReach + 1)) / 2)
                                                                        : nx - 2 * kReach) *
                             (double)(ny - 2 * kReach);
    const double moved = pattern == RLBM_PROBE_READ   ? (double)bytes
                         : pattern == RLBM_PROBE_COPY ? 2.0 * (double)bytes
                                                      : 2.0 * kQ * elem_bytes * interior;
    if (gbs) *gbs = moved / t / 1e9;
    if (us) *us = t * 1e6;
    return RLBM_OK;
}
