// gfx950 kernels of the fused relativistic LB step.
//
// Storage: 48 SoA planes of nx*ny values, plane i = population i = 4*d + j,
// holding the post-collision state f*(t) as the scaled deviation eta_i from
// the reference rest equilibrium.  One step reads f*(t) from src and writes
// f*(t+1) to dst (ping-pong), so every stored value is read exactly once
// and written exactly once per step: the step is bound by HBM bandwidth.
//
// Work mapping: one thread per site; a block covers tile_x consecutive
// sites of `rows` rows, so each wavefront reads 64 consecutive values of a
// plane row (shifted by the hop) and writes 64 aligned values.  Blocks whose
// 5-site halo lies inside the lattice (and without a solid mask) take a
// branch-free gather; the others resolve periodic wrap, contact ghost spans
// and bounce-back per population.
#include "rlbm_kernels.h"

namespace rlbm {
namespace {

template <class S>
struct StoreIO;
template <>
struct StoreIO<double> {
    template <class R>
    __device__ static R load(const double *p) { return R(*p); }
    template <class R>
    __device__ static void store(double *p, R v) { *p = double(v); }
    template <class R>
    __device__ static void store_nt(double *p, R v) { __builtin_nontemporal_store(double(v), p); }
};
template <>
struct StoreIO<float> {
    template <class R>
    __device__ static R load(const float *p) { return R(*p); }
    template <class R>
    __device__ static void store(float *p, R v) { *p = float(v); }
    template <class R>
    __device__ static void store_nt(float *p, R v) { __builtin_nontemporal_store(float(v), p); }
};
template <>
struct StoreIO<_Float16> {
    template <class R>
    __device__ static R load(const _Float16 *p) { return R(float(*p)); }
    template <class R>
    __device__ static void store(_Float16 *p, R v) { *p = _Float16(float(v)); }
    template <class R>
    __device__ static void store_nt(_Float16 *p, R v) { __builtin_nontemporal_store(_Float16(float(v)), p); }
};

struct SiteFields {
    double n, vx, vy, eps;
};

// Collision of one site, in place on the 48 scaled deviations h.
// Steps: moments -> Landau frame -> n, T -> Appendix B projections ->
// equilibrium and forcing polynomials -> relaxation with
// omega_d = p_i.U / (p0_i tau) = (U^0 - nhat_d . U_s) / tau.
template <class R>
__device__ __forceinline__ bool collide_site(R (&h)[kQ], const StepArgs<R> &A, SiteFields &out, R fx, R fy,
                                             bool has_force)
{
    // ---- moments of the deviation, one pair of opposite directions at a time ----
    R N0 = 0, Nx = 0, Ny = 0, T00 = 0, T0x = 0, T0y = 0, Txx = 0, Txy = 0, Tyy = 0;
#pragma unroll
    for (int d = 0; d < kDirs / 2; ++d) {
        const int g = kGroup[d];
        R a1 = 0, a2 = 0, b1 = 0, b2 = 0;
#pragma unroll
        for (int j = 0; j < kShells; ++j) {
            a1 += A.wp0[g][j] * h[4 * d + j];
            a2 += A.wp0[g][j] * h[4 * (d + 6) + j];
            b1 += A.wp0sq[g][j] * h[4 * d + j];
            b2 += A.wp0sq[g][j] * h[4 * (d + 6) + j];
        }
        const DirTrig tg = dir_trig(d);
        const R c = R(tg.c), s = R(tg.s);
        const R Ae = a1 + a2, Ao = a1 - a2, Be = b1 + b2, Bo = b1 - b2;
        N0 += Ae;
        Nx += Ao * c;
        Ny += Ao * s;
        T00 += Be;
        T0x += Bo * c;
        T0y += Bo * s;
        Txx += Be * (c * c);
        Txy += Be * (c * s);
        Tyy += Be * (s * s);
    }
    // ---- Landau frame in float64, reference moments added back ----
    const double nT = A.n_ref * A.T_ref;
    const double dN0 = A.n_ref + double(N0), dNx = double(Nx), dNy = double(Ny);
    double eps, u0, ux, uy;
    const bool ok = landau_frame(2.0 * nT + double(T00), double(T0x), double(T0y), nT + double(Txx), double(Txy),
                                 nT + double(Tyy), eps, u0, ux, uy);
    const double n = u0 * dN0 - ux * dNx - uy * dNy;
    const double T = eps / (2.0 * n);
    out.n = n;
    out.vx = ux / u0;
    out.vy = uy / u0;
    out.eps = eps;
    // ---- equilibrium and force coefficients (deviation from the reference, / scale) ----
    double a[kK];
    appendix_b(n, T, u0, ux, uy, a);
    R ad[kK];
#pragma unroll
    for (int k = 0; k < kK; ++k) ad[k] = R((a[k] - A.a_ref[k]) * A.inv_scale);
    R Ha[kK], Hb[kK];
    appendix_a_to_harmonics(ad, Ha);
    if (has_force) {
        // b = (Fx C_x + Fy C_y) a / scale with a / scale = ad + a_ref / scale
        R as[kK];
#pragma unroll
        for (int k = 0; k < kK; ++k) as[k] = ad[k];
#pragma unroll
        for (int r = 0; r < 4; ++r) as[kRestK[r]] += A.aref_s[r];
        R bx[kK], by[kK], b[kK];
#pragma unroll
        for (int k = 0; k < kK; ++k) bx[k] = by[k] = R(0);
        if (fx != R(0)) {
#pragma unroll
            for (int q = 0; q < kForceNx; ++q) bx[kForceX[q].k] += R(kForceX[q].v) * as[kForceX[q].m];
        }
        if (fy != R(0)) {
#pragma unroll
            for (int q = 0; q < kForceNy; ++q) by[kForceY[q].k] += R(kForceY[q].v) * as[kForceY[q].m];
        }
#pragma unroll
        for (int k = 0; k < kK; ++k) b[k] = fx * bx[k] + fy * by[k];
        appendix_a_to_harmonics(b, Hb);
    } else {
#pragma unroll
        for (int k = 0; k < kK; ++k) Hb[k] = R(0);
    }
    // ---- relaxation plus forcing, one pair of opposite directions at a time ----
    const R U0 = R(u0 * A.tau_inv), Ux = R(ux * A.tau_inv), Uy = R(uy * A.tau_inv);
#pragma unroll
    for (int d = 0; d < kDirs / 2; ++d) {
        const DirTrig tg = dir_trig(d);
        R Ea[4], Oa[4], Eb[4], Ob[4];
        harmonics_pair(Ha, tg, Ea, Oa);
        harmonics_pair(Hb, tg, Eb, Ob);
        const R proj = Ux * R(tg.c) + Uy * R(tg.s);
        const R wp = U0 - proj, wm = U0 + proj;  // omega of d and of d + 6
        R Gp[4], Gm[4];
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            Gp[e] = wp * (Ea[e] + Oa[e]) - (Eb[e] + Ob[e]);
            Gm[e] = wm * (Ea[e] - Oa[e]) - (Eb[e] - Ob[e]);
        }
#pragma unroll
        for (int j = 0; j < kShells; ++j) {
            const R p = A.p0[j];
            const R qp = ((Gp[3] * p + Gp[2]) * p + Gp[1]) * p + Gp[0];
            const R qm = ((Gm[3] * p + Gm[2]) * p + Gm[1]) * p + Gm[0];
            h[4 * d + j] = (R(1) - wp) * h[4 * d + j] + qp;
            h[4 * (d + 6) + j] = (R(1) - wm) * h[4 * (d + 6) + j] + qm;
        }
    }
    return ok;
}

template <class R>
__device__ __forceinline__ void write_fields(const StepArgs<R> &A, long long site, const SiteFields &f, bool ok)
{
    if (!ok) {
        A.fn[site] = NAN;
        A.fvx[site] = NAN;
        A.fvy[site] = NAN;
        A.feps[site] = NAN;
        return;
    }
    A.fn[site] = f.n;
    A.fvx[site] = f.vx;
    A.fvy[site] = f.vy;
    A.feps[site] = f.eps;
}

// Density of the previous state at (x, y) for the local-capacitance gradient
// at (x0, y0): periodic wrap, else an off-lattice or solid neighbour takes
// the density of the site itself.
template <class R>
__device__ __forceinline__ double lca_density(const StepArgs<R> &A, int x, int y, long long site0)
{
    if (A.periodic_x) x = x < 0 ? x + A.nx : (x >= A.nx ? x - A.nx : x);
    if (A.periodic_y) y = y < 0 ? y + A.ny : (y >= A.ny ? y - A.ny : y);
    if ((unsigned)x >= (unsigned)A.nx || (unsigned)y >= (unsigned)A.ny) return A.n_prev[site0];
    const long long s = (long long)y * A.nx + x;
    if (A.has_mask && A.mask[s]) return A.n_prev[site0];
    return A.n_prev[s];
}

// Total force on a site with the local-capacitance term: drive minus
// inv_cg times the central-difference gradient of the previous density.
// `inner`: the four neighbours lie on the lattice and none is solid.
template <class R>
__device__ __forceinline__ void lca_force(const StepArgs<R> &A, int x, int y, long long site, bool inner, R &fx,
                                          R &fy)
{
    double ge, gw, gn, gs;
    if (inner) {
        ge = A.n_prev[site + 1];
        gw = A.n_prev[site - 1];
        gn = A.n_prev[site + A.nx];
        gs = A.n_prev[site - A.nx];
    } else {
        ge = lca_density(A, x + 1, y, site);
        gw = lca_density(A, x - 1, y, site);
        gn = lca_density(A, x, y + 1, site);
        gs = lca_density(A, x, y - 1, site);
    }
    const double gx = 0.5 * (ge - gw), gy = 0.5 * (gn - gs);
    fx = R(double(A.fx) - A.inv_cg * gx);
    fy = R(double(A.fy) - A.inv_cg * gy);
}

// Gather of one site with the boundary rules: periodic wrap, then a contact's
// ghost span (fixed equilibrium), otherwise bounce-back from the site itself
// (also for a solid source site).
template <class S, class R>
__device__ __forceinline__ void gather_general(const StepArgs<R> &A, const S *__restrict__ src, int x, int y,
                                               long long site, R (&h)[kQ])
{
    const int nx = A.nx, ny = A.ny;
    const long long P = A.plane;
#pragma unroll
    for (int i = 0; i < kQ; ++i) {
        const int d = i / kShells;
        const int o = kShells * ((d + kDirs / 2) % kDirs) + (i % kShells);
        int sx = x - kCx[d], sy = y - kCy[d];
        if (A.periodic_x) {
            while (sx < 0) sx += nx;
            while (sx >= nx) sx -= nx;
        }
        if (A.periodic_y) {
            while (sy < 0) sy += ny;
            while (sy >= ny) sy -= ny;
        }
        const bool inside = (unsigned)sx < (unsigned)nx && (unsigned)sy < (unsigned)ny;
        const long long s2 = (long long)sy * nx + sx;
        const bool pull = inside && !(A.has_mask && A.mask[s2]);
        R v;
        if (pull) {
            v = StoreIO<S>::template load<R>(src + (long long)i * P + s2);
        } else {
            int c = -1;
            if (!inside) {
                if (sy < 0 && (unsigned)sx < (unsigned)nx)
                    c = A.edge_contact[sx];
                else if (sy >= ny && (unsigned)sx < (unsigned)nx)
                    c = A.edge_contact[nx + sx];
                else if (sx < 0 && (unsigned)sy < (unsigned)ny)
                    c = A.edge_contact[2 * nx + sy];
                else if (sx >= nx && (unsigned)sy < (unsigned)ny)
                    c = A.edge_contact[2 * nx + ny + sy];
            }
            v = c >= 0 ? A.contact_eta[c * kQ + i] : StoreIO<S>::template load<R>(src + (long long)o * P + site);
        }
        h[i] = v;
    }
}

// One block of a time step.  The step's 1-D grid of 256-thread blocks: the
// first nbnd blocks take the boundary sites (gather table or computed
// gather), the rest tile the interior x in [5, nx - 5), y in [5, ny - 5)
// with tile_x * rows sites per block, tiles aligned to tile_x so every
// wavefront stores 64 aligned values.
template <class S, class R, bool LCA>
__device__ __forceinline__ void step_block(const StepArgs<R> &A, const S *__restrict__ src, S *__restrict__ dst,
                                           int b, int nbnd, int tile_x, int tiles_x, int all, int wf)
{
    const int t = threadIdx.x;
    const int nx = A.nx;
    const long long P = A.plane;
    int x, y;
    bool inner;
    R h[kQ];
    if (b < nbnd) {
        const long long idx = (long long)b * blockDim.x + t;
        if (idx >= boundary_count(nx, A.ny, all)) return;
        boundary_site(idx, nx, A.ny, all, x, y);
        inner = false;
        const long long site = (long long)y * nx + x;
        if (A.has_mask && A.mask[site]) {
            if (wf) {
                A.fn[site] = 0.0;
                A.fvx[site] = 0.0;
                A.fvy[site] = 0.0;
                A.feps[site] = 0.0;
            }
            return;
        }
        if (A.gather_tab) {
            const unsigned *__restrict__ tab = A.gather_tab;
#pragma unroll
            for (int i = 0; i < kQ; ++i) {
                const unsigned c = tab[(long long)i * A.nbnd + idx];
                h[i] = (c & kContactFlag) ? A.contact_eta[c & ~kContactFlag]
                                          : StoreIO<S>::template load<R>(src + c);
            }
        } else {
            gather_general<S, R>(A, src, x, y, site, h);
        }
    } else {
        const int tb = b - nbnd;
        const int by = tb / tiles_x, bx = tb - by * tiles_x;
        const int rows = blockDim.x / tile_x;
        const int ty = t / tile_x;
        x = bx * tile_x + (t - ty * tile_x);
        y = kReach + by * rows + ty;
        if (x < kReach || x >= nx - kReach || y >= A.ny - kReach) return;
        inner = true;
        // uniform plane base pointers + one 32-bit site offset
        const unsigned site = (unsigned)y * (unsigned)nx + (unsigned)x;
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            const int d = i / kShells;
            const S *__restrict__ plane = src + ((long long)i * P - ((long long)kCy[d] * nx + kCx[d]));
            h[i] = StoreIO<S>::template load<R>(plane + site);
        }
    }
    const unsigned site = (unsigned)y * (unsigned)nx + (unsigned)x;
    SiteFields f;
    bool ok;
    if constexpr (LCA) {
        R fx, fy;
        lca_force(A, x, y, site, inner, fx, fy);
        ok = collide_site<R>(h, A, f, fx, fy, true);
        A.n_next[site] = ok ? f.n : NAN;
    } else {
        (void)inner;
        ok = collide_site<R>(h, A, f, A.fx, A.fy, A.has_force != 0);
    }
    if (wf) write_fields(A, site, f, ok);
    if (A.nt_store) {
        // streaming stores: the next step reads these values once, from HBM
#pragma unroll
        for (int i = 0; i < kQ; ++i) StoreIO<S>::template store_nt<R>(dst + (long long)i * P + site, h[i]);
    } else {
#pragma unroll
        for (int i = 0; i < kQ; ++i) {
            S *__restrict__ plane = dst + (long long)i * P;
            StoreIO<S>::template store<R>(plane + site, h[i]);
        }
    }
}

template <class S, class R, bool LCA>
__global__ __launch_bounds__(256) void step_kernel(const StepArgs<R> A, const S *__restrict__ src,
                                                   S *__restrict__ dst, int nbnd, int tile_x, int tiles_x, int all)
{
    step_block<S, R, LCA>(A, src, dst, blockIdx.x, nbnd, tile_x, tiles_x, all, A.write_fields);
}

// Batched step: a persistent grid drains the work list of (sample, block)
// items through an atomic counter; each item is one block of that sample's
// step grid.  The last block to leave resets the counters, so the next launch
// (or graph replay) starts from zero without a memset.
template <class S, class R>
__global__ __launch_bounds__(256) void batch_step_kernel(const BatchDesc<R> *__restrict__ descs,
                                                         const unsigned *__restrict__ items,
                                                         const int *__restrict__ n_items_p,
                                                         unsigned *__restrict__ counters, int parity, int wf)
{
    __shared__ unsigned s_item;
    const unsigned n_items = (unsigned)*n_items_p;
    for (;;) {
        if (threadIdx.x == 0) s_item = atomicAdd(&counters[0], 1u);
        __syncthreads();
        const unsigned k = s_item;
        __syncthreads();
        if (k >= n_items) break;
        const unsigned it = __builtin_amdgcn_readfirstlane(items[k]);
        const int smp = (int)(it >> kItemBlockBits), b = (int)(it & ((1u << kItemBlockBits) - 1));
        const BatchDesc<R> &D = descs[smp];
        const int par = parity ^ D.parity_xor;
        step_block<S, R, false>(D.a, static_cast<const S *>(D.pop[par]), static_cast<S *>(D.pop[par ^ 1]), b, D.nbnd,
                                D.tile_x, D.tiles_x, D.all, wf);
    }
    if (threadIdx.x == 0) {
        __threadfence();
        const unsigned done = atomicAdd(&counters[1], 1u);
        if (done == gridDim.x - 1) {
            atomicExch(&counters[0], 0u);
            atomicExch(&counters[1], 0u);
        }
    }
}

// Per-sample residual partial sums: block (s, j) covers sites j, j + B*256,
// ... of sample s; part[(s * B + j) * 3 + {0,1,2}] = |u - u_prev|^2, |u|^2,
// unhealthy count.
template <class R>
__global__ __launch_bounds__(256) void batch_residual_kernel(const BatchDesc<R> *__restrict__ descs,
                                                             double *__restrict__ part)
{
    const int smp = blockIdx.y, B = gridDim.x;
    const BatchDesc<R> &D = descs[smp];
    const long long n = D.a.plane;
    double dv = 0.0, vv = 0.0, bad = 0.0;
    for (long long s = (long long)blockIdx.x * blockDim.x + threadIdx.x; s < n; s += (long long)B * blockDim.x) {
        if (D.a.has_mask && D.a.mask[s]) continue;
        const double a = D.a.fvx[s], b = D.a.fvy[s], dn = D.a.fn[s];
        const double ex = a - D.pvx[s], ey = b - D.pvy[s];
        const double v2 = a * a + b * b;
        if (!(dn > 0.0) || !(v2 < 1.0) || !isfinite(a) || !isfinite(b) || !isfinite(dn)) bad += 1.0;
        dv += ex * ex + ey * ey;
        vv += v2;
    }
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
        double *o = part + ((long long)smp * B + blockIdx.x) * 3;
        o[0] = s0;
        o[1] = s1;
        o[2] = s2;
    }
}

template <class S, class R>
__global__ __launch_bounds__(256) void init_kernel(const StepArgs<R> A, const double *__restrict__ n_in,
                                                   const double *__restrict__ T_in, const double *__restrict__ vx_in,
                                                   const double *__restrict__ vy_in, double un, double uT, double uvx,
                                                   double uvy, S *__restrict__ dst, int mode)
{
    const long long site = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= A.plane) return;
    if (A.has_mask && A.mask[site]) {
        if (mode == kInitDensity) return;
        for (int i = 0; i < kQ; ++i) StoreIO<S>::template store<R>(dst + (long long)i * A.plane + site, R(0));
        A.fn[site] = 0.0;
        A.fvx[site] = 0.0;
        A.fvy[site] = 0.0;
        A.feps[site] = 0.0;
        return;
    }
    const double n = n_in ? n_in[site] : un;
    const double T = T_in ? T_in[site] : uT;
    const double vx = vx_in ? vx_in[site] : uvx;
    const double vy = vy_in ? vy_in[site] : uvy;
    const double g = 1.0 / sqrt(1.0 - vx * vx - vy * vy);
    double a[kK];
    appendix_b(n, T, g, g * vx, g * vy, a);
    R ad[kK], H[kK];
    for (int k = 0; k < kK; ++k) ad[k] = R((a[k] - A.a_ref[k]) * A.inv_scale);
    appendix_a_to_harmonics(ad, H);
    R h[kQ];
#pragma unroll
    for (int d = 0; d < kDirs / 2; ++d) {
        R E[4], O[4];
        harmonics_pair(H, dir_trig(d), E, O);
#pragma unroll
        for (int j = 0; j < kShells; ++j) {
            const R p = A.p0[j];
            h[4 * d + j] = (((E[3] + O[3]) * p + (E[2] + O[2])) * p + (E[1] + O[1])) * p + (E[0] + O[0]);
            h[4 * (d + 6) + j] = (((E[3] - O[3]) * p + (E[2] - O[2])) * p + (E[1] - O[1])) * p + (E[0] - O[0]);
        }
    }
    SiteFields f;
    R fx = A.fx, fy = A.fy;
    bool force = A.has_force != 0;
    if (mode == kInitLca) {
        const int y = (int)(site / A.nx), x = (int)(site - (long long)y * A.nx);
        lca_force(A, x, y, site, false, fx, fy);
        force = true;
    }
    const bool ok = collide_site<R>(h, A, f, fx, fy, force);
    if (mode == kInitDensity) {
        A.n_next[site] = ok ? f.n : NAN;
        return;
    }
    write_fields(A, site, f, ok);
    for (int i = 0; i < kQ; ++i) StoreIO<S>::template store<R>(dst + (long long)i * A.plane + site, h[i]);
}

template <class S>
__global__ __launch_bounds__(256) void decode_kernel(long long plane, const S *__restrict__ src,
                                                     const double *__restrict__ fref,
                                                     const double *__restrict__ wscale, double *__restrict__ f)
{
    const long long site = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (site >= plane) return;
    for (int i = 0; i < kQ; ++i) {
        const double e = StoreIO<S>::template load<double>(src + (long long)i * plane + site);
        f[(long long)i * plane + site] = fref[i] + wscale[i] * e;
    }
}

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

template <class S, class R>
hipError_t launch_step_t(const void *args, const void *src, void *dst, LaunchShape sh, hipStream_t s)
{
    const StepArgs<R> &A = *static_cast<const StepArgs<R> *>(args);
    const bool interior = !A.has_mask && A.nx > 2 * kReach && A.ny > 2 * kReach;
    const int block = 256;
    const long long nb = boundary_count(A.nx, A.ny, !interior);
    const int nbnd = (int)((nb + block - 1) / block);
    int tiles_x = 0, tiles = 0;
    if (interior) {
        const int rows = block / sh.tile_x;
        tiles_x = (A.nx + sh.tile_x - 1) / sh.tile_x;
        tiles = tiles_x * ((A.ny - 2 * kReach + rows - 1) / rows);
    }
    if (A.n_prev)
        hipLaunchKernelGGL((step_kernel<S, R, true>), dim3((unsigned)(nbnd + tiles)), dim3(block), 0, s, A,
                           static_cast<const S *>(src), static_cast<S *>(dst), nbnd, sh.tile_x, tiles_x,
                           interior ? 0 : 1);
    else
        hipLaunchKernelGGL((step_kernel<S, R, false>), dim3((unsigned)(nbnd + tiles)), dim3(block), 0, s, A,
                           static_cast<const S *>(src), static_cast<S *>(dst), nbnd, sh.tile_x, tiles_x,
                           interior ? 0 : 1);
    return hipGetLastError();
}

template <class S, class R>
hipError_t launch_init_t(const void *args, const double *n, const double *T, const double *vx, const double *vy,
                         const double u[4], void *dst, int mode, hipStream_t s)
{
    const StepArgs<R> &A = *static_cast<const StepArgs<R> *>(args);
    if ((mode == kInitDensity && !A.n_next) || (mode == kInitLca && !A.n_prev) || mode < 0 || mode > 2)
        return hipErrorInvalidValue;
    const int block = 256;
    const long long grid = (A.plane + block - 1) / block;
    hipLaunchKernelGGL((init_kernel<S, R>), dim3((unsigned)grid), dim3(block), 0, s, A, n, T, vx, vy, u[0], u[1], u[2],
                       u[3], static_cast<S *>(dst), mode);
    return hipGetLastError();
}

template <class S, class R>
hipError_t launch_batch_t(const void *descs, const unsigned *items, const int *n_items, unsigned *counters, int grid,
                          int parity, int wf, hipStream_t s)
{
    hipLaunchKernelGGL((batch_step_kernel<S, R>), dim3(grid), dim3(256), 0, s,
                       static_cast<const BatchDesc<R> *>(descs), items, n_items, counters, parity, wf);
    return hipGetLastError();
}

template <class S, class R>
int batch_grid_t()
{
    int dev = 0, per_cu = 0;
    hipDeviceProp_t prop;
    if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) return 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, batch_step_kernel<S, R>, 256, 0) != hipSuccess) return 0;
    return per_cu * prop.multiProcessorCount;
}

}  // namespace

hipError_t launch_batch_step(Store st, const void *descs, const unsigned *items, const int *n_items,
                             unsigned *counters, int grid, int parity, int write_fields, hipStream_t s)
{
    switch (st) {
    case Store::F64: return launch_batch_t<double, double>(descs, items, n_items, counters, grid, parity, write_fields, s);
    case Store::F32: return launch_batch_t<float, float>(descs, items, n_items, counters, grid, parity, write_fields, s);
    case Store::F16:
        return launch_batch_t<_Float16, float>(descs, items, n_items, counters, grid, parity, write_fields, s);
    }
    return hipErrorInvalidValue;
}

int batch_resident_blocks(Store st)
{
    switch (st) {
    case Store::F64: return batch_grid_t<double, double>();
    case Store::F32: return batch_grid_t<float, float>();
    case Store::F16: return batch_grid_t<_Float16, float>();
    }
    return 0;
}

hipError_t launch_batch_residual(Store st, const void *descs, int nsamples, int blocks_per_sample, double *part,
                                 hipStream_t s)
{
    const dim3 grid(blocks_per_sample, nsamples);
    if (st == Store::F64)
        hipLaunchKernelGGL(batch_residual_kernel<double>, grid, dim3(256), 0, s,
                           static_cast<const BatchDesc<double> *>(descs), part);
    else
        hipLaunchKernelGGL(batch_residual_kernel<float>, grid, dim3(256), 0, s,
                           static_cast<const BatchDesc<float> *>(descs), part);
    return hipGetLastError();
}

hipError_t launch_step(Store st, const void *args, const void *src, void *dst, LaunchShape shape, hipStream_t s)
{
    if (shape.tile_x <= 0 || shape.rows <= 0 || shape.tile_x * shape.rows != 256 || shape.tile_x % 64)
        return hipErrorInvalidValue;
    switch (st) {
    case Store::F64: return launch_step_t<double, double>(args, src, dst, shape, s);
    case Store::F32: return launch_step_t<float, float>(args, src, dst, shape, s);
    case Store::F16: return launch_step_t<_Float16, float>(args, src, dst, shape, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_init(Store st, const void *args, const double *n, const double *T, const double *vx,
                       const double *vy, const double u[4], void *dst, int mode, hipStream_t s)
{
    switch (st) {
    case Store::F64: return launch_init_t<double, double>(args, n, T, vx, vy, u, dst, mode, s);
    case Store::F32: return launch_init_t<float, float>(args, n, T, vx, vy, u, dst, mode, s);
    case Store::F16: return launch_init_t<_Float16, float>(args, n, T, vx, vy, u, dst, mode, s);
    }
    return hipErrorInvalidValue;
}

hipError_t launch_decode(Store st, int nx, int ny, const void *src, const double *fref, const double *wscale,
                         double *f, hipStream_t s)
{
    const long long plane = (long long)nx * ny;
    const int block = 256;
    const dim3 grid((unsigned)((plane + block - 1) / block));
    switch (st) {
    case Store::F64:
        hipLaunchKernelGGL(decode_kernel<double>, grid, dim3(block), 0, s, plane, (const double *)src, fref, wscale, f);
        break;
    case Store::F32:
        hipLaunchKernelGGL(decode_kernel<float>, grid, dim3(block), 0, s, plane, (const float *)src, fref, wscale, f);
        break;
    case Store::F16:
        hipLaunchKernelGGL(decode_kernel<_Float16>, grid, dim3(block), 0, s, plane, (const _Float16 *)src, fref,
                           wscale, f);
        break;
    }
    return hipGetLastError();
}

hipError_t launch_residual(int nsites, const unsigned char *mask, const double *n, const double *vx, const double *vy,
                           const double *pvx, const double *pvy, double *part, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(residual_kernel, dim3(nblocks), dim3(256), 0, s, nsites, mask, n, vx, vy, pvx, pvy, part);
    return hipGetLastError();
}

}  // namespace rlbm
