// Dispatch of the step kernels by storage (each storage's kernels live in a
// translation unit of their own: step_f64.hip, step_f32.hip, step_f16.hip)
// and the storage-independent residual kernel.
#include <mutex>

#include "rlbm_kernels.h"

namespace rlbm {

#define RLBM_DECLARE_STORAGE_LAUNCHERS(SUFFIX)                                                                     \
    hipError_t launch_step_##SUFFIX(const void *args, const void *src, void *dst, LaunchShape sh, hipStream_t s); \
    hipError_t launch_init_##SUFFIX(const void *args, const double *n, const double *T, const double *vx,          \
                                    const double *vy, const double u[4], void *dst, int mode, hipStream_t s);      \
    hipError_t launch_batch_##SUFFIX(const void *descs, const unsigned *items, const int *n_items, int grid,       \
                                     int parity, int wf, int xcd, int nt, hipStream_t s);                          \
    hipError_t launch_batch_residual_##SUFFIX(const void *descs, int nsamples, int blocks_per_sample,              \
                                              double *part, hipStream_t s);                                        \
    hipError_t launch_decode_##SUFFIX(long long plane, const void *src, const double *fref, const double *wscale,  \
                                      double *f, hipStream_t s);
RLBM_DECLARE_STORAGE_LAUNCHERS(f64)
RLBM_DECLARE_STORAGE_LAUNCHERS(f32)
RLBM_DECLARE_STORAGE_LAUNCHERS(f16)
#undef RLBM_DECLARE_STORAGE_LAUNCHERS

namespace {

__global__ __launch_bounds__(256) void residual_kernel(int nsites, const unsigned char *__restrict__ mask,
                                                       const double *__restrict__ n, const double *__restrict__ vx,
                                                       const double *__restrict__ vy, const double *__restrict__ pvx,
                                                       const double *__restrict__ pvy, double *__restrict__ part)
{
    double dv = 0.0, vv = 0.0, bad = 0.0;
    for (int s = blockIdx.x * blockDim.x + threadIdx.x; s < nsites; s += gridDim.x * blockDim.x) {
        if (mask && mask[s]) continue;
        const double a = vx[s], b = vy[s], dn = n[s];
        const double ex = a - pvx[s], ey = b - pvy[s];
        const double v2 = a * a + b * b;
        if (!(dn > 0.0) || !(v2 < 1.0) || !isfinite(a) || !isfinite(b) || !isfinite(dn)) bad += 1.0;
        dv += ex * ex + ey * ey;
        vv += v2;
    }
    // wavefront reduction (64 lanes), then across the block's wavefronts
    for (int off = 32; off > 0; off >>= 1) {
        dv += __shfl_down(dv, off, 64);
        vv += __shfl_down(vv, off, 64);
        bad += __shfl_down(bad, off, 64);
    }
    __shared__ double red[3][256 / 64];
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (lane == 0) {
        red[0][wid] = dv;
        red[1][wid] = vv;
        red[2][wid] = bad;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double s0 = 0, s1 = 0, s2 = 0;
        for (int w = 0; w < (int)(blockDim.x / 64); ++w) {
            s0 += red[0][w];
            s1 += red[1][w];
            s2 += red[2][w];
        }
        part[3 * blockIdx.x + 0] = s0;
        part[3 * blockIdx.x + 1] = s1;
        part[3 * blockIdx.x + 2] = s2;
    }
}

}  // namespace

hipError_t launch_batch_step(Store st, const void *descs, const unsigned *items, const int *n_items, int grid,
                             int parity, int write_fields, int xcd, int nt, hipStream_t s)
{
    if (grid <= 0) return hipErrorInvalidValue;
    switch (st) {
    case Store::F64: return launch_batch_f64(descs, items, n_items, grid, parity, write_fields, xcd, nt, s);
    case Store::F32: return launch_batch_f32(descs, items, n_items, grid, parity, write_fields, xcd, nt, s);
    case Store::F16: return launch_batch_f16(descs, items, n_items, grid, parity, write_fields, xcd, nt, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_batch_residual(Store st, const void *descs, int nsamples, int blocks_per_sample, double *part,
                                 hipStream_t s)
{
    switch (st) {
    case Store::F64: return launch_batch_residual_f64(descs, nsamples, blocks_per_sample, part, s);
    case Store::F32: return launch_batch_residual_f32(descs, nsamples, blocks_per_sample, part, s);
    case Store::F16: return launch_batch_residual_f16(descs, nsamples, blocks_per_sample, part, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_step(Store st, const void *args, const void *src, void *dst, LaunchShape shape, hipStream_t s)
{
    if (shape.tile_x <= 0 || shape.rows <= 0 || shape.tile_x * shape.rows != 256 || shape.tile_x % 64 ||
        (shape.xcd != 0 && shape.xcd != 1))
        return hipErrorInvalidValue;
    switch (st) {
    case Store::F64: return launch_step_f64(args, src, dst, shape, s);
    case Store::F32: return launch_step_f32(args, src, dst, shape, s);
    case Store::F16: return launch_step_f16(args, src, dst, shape, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_init(Store st, const void *args, const double *n, const double *T, const double *vx,
                       const double *vy, const double u[4], void *dst, int mode, hipStream_t s)
{
    switch (st) {
    case Store::F64: return launch_init_f64(args, n, T, vx, vy, u, dst, mode, s);
    case Store::F32: return launch_init_f32(args, n, T, vx, vy, u, dst, mode, s);
    case Store::F16: return launch_init_f16(args, n, T, vx, vy, u, dst, mode, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_decode(Store st, int nx, int ny, const void *src, const double *fref, const double *wscale,
                         double *f, hipStream_t s)
{
    const long long plane = (long long)nx * ny;
    switch (st) {
    case Store::F64: return launch_decode_f64(plane, src, fref, wscale, f, s);
    case Store::F32: return launch_decode_f32(plane, src, fref, wscale, f, s);
    case Store::F16: return launch_decode_f16(plane, src, fref, wscale, f, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_residual(int nsites, const unsigned char *mask, const double *n, const double *vx, const double *vy,
                           const double *pvx, const double *pvy, double *part, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(residual_kernel, dim3(nblocks), dim3(256), 0, s, nsites, mask, n, vx, vy, pvx, pvy, part);
    return hipGetLastError();
}

// ---- residual without allocation ----
//
// The per-block partial sums of residual_kernel and their three totals live
// in this file-scope array instead of a buffer the library allocates: one
// copy per device, held until the process ends and shared by every call on
// that device (calls that overlap on one device race).  Each call overwrites
// the partial sums it reads and the totals, so nothing needs clearing.
static __device__ __align__(256) double scratch[3 * kNoAllocResidualBlocks + 3];

namespace {

// The device address of `scratch`, per device (the array's name in host code
// only stands in for it), looked up on the first call on each device.
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
double *g_scratch[kMaxDevices] = {};

hipError_t scratch_of_current_device(double **out)
{
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return hipSuccess;
}

// One thread adds the partial sums in block order, as the host loop of the
// allocating residual does, so both give the same totals bit for bit.
__global__ __launch_bounds__(64) void residual_total_kernel(const double *__restrict__ part, int nblocks,
                                                            double *__restrict__ out)
{
    if (threadIdx.x != 0) return;
    double dv = 0.0, vv = 0.0, bad = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        dv += part[3 * b];
        vv += part[3 * b + 1];
        bad += part[3 * b + 2];
    }
    out[0] = dv;
    out[1] = vv;
    out[2] = bad;
}

}  // namespace

hipError_t launch_residual_noalloc(int nsites, const unsigned char *mask, const double *n, const double *vx,
                                   const double *vy, const double *pvx, const double *pvy, int nblocks,
                                   double totals[3], hipStream_t s)
{
    if (nblocks < 1 || nblocks > kNoAllocResidualBlocks || !totals) return hipErrorInvalidValue;
    double *ptr = nullptr;
    hipError_t e = scratch_of_current_device(&ptr);
    if (e != hipSuccess) return e;
    double *tot = ptr + 3 * kNoAllocResidualBlocks;
    hipLaunchKernelGGL(residual_kernel, dim3(nblocks), dim3(256), 0, s, nsites, mask, n, vx, vy, pvx, pvy, ptr);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(residual_total_kernel, dim3(1), dim3(64), 0, s, ptr, nblocks, tot);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = hipMemcpyAsync(totals, tot, 3 * sizeof(double), hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

}  // namespace rlbm
